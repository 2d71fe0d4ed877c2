// Sweep kernels of the JGS2 per-iteration solve (gfx950).
//
// Thread mapping: 32 lanes per vertex sub-problem, 8 vertices per 256-thread
// block.  A vertex's lanes split its incident tets (a Kuhn mesh has at most
// 24), its one-ring rows and its cubature samples, then combine with a
// 5-step xor butterfly, so no floating-point atomics are used and every
// result is bitwise deterministic.  Blocks are remapped so that each XCD
// (blocks are dealt round-robin to the 8 XCDs) works on one contiguous
// range of vertices, keeping a slab's tets and neighbours in that XCD's L2.
//
// Vertex data are float4 records (one 16-byte load per gathered corner):
// displacement u = x - X from the rest shape (so H = F - I keeps full FP32
// precision and the stress is evaluated from H without cancelling O(mu)
// terms), inertial target with m/h^2 in w, gradient, and the per-vertex
// rotation as a unit quaternion.
#include <hip/hip_ext.h>

#include <hip/hip_cooperative_groups.h>

#include "jgs2_internal.h"
#include "jgs2_math.h"

namespace jgs2 {

// ---------------------------------------------------------------------------
// Index checks of the bounds-checked build (compiled with JGS2_BOUNDS_CHECK).
// An index read from a table (a list entry, a vertex or tet id, a position,
// a one-ring slot, a super-tile id or a partial range) is checked against
// its buffer's extent before use.  The first failure's source line, value
// and extent go to the handle's record; the index is replaced by 0 so that
// the access stays inside the buffer.  In other builds ix() is the index.
// ---------------------------------------------------------------------------
#ifdef JGS2_BOUNDS_CHECK
__device__ __noinline__ void bounds_fail(unsigned long long* rec, long long i, long long n, int site) {
    if (atomicCAS(rec, 0ull, (unsigned long long)site) == 0ull) {
        rec[1] = (unsigned long long)i;
        rec[2] = (unsigned long long)n;
    }
}
#endif

__device__ __forceinline__ int ix(const SweepArgs& a, long long i, long long n, int site) {
#ifdef JGS2_BOUNDS_CHECK
    if ((unsigned long long)i >= (unsigned long long)n) {
        if (a.bounds) bounds_fail(a.bounds, i, n, site);
        return 0;
    }
#else
    (void)a; (void)n; (void)site;
#endif
    return (int)i;
}
#define IX(a, i, n) ix((a), (i), (n), __LINE__)

// An incidence entry (tet << 2 | corner, three corner vertex ids), checked.
__device__ __forceinline__ int4 ix_inc(const SweepArgs& a, int4 e, int site) {
#ifdef JGS2_BOUNDS_CHECK
    e.x = (ix(a, e.x >> 2, a.nT, site) << 2) | (e.x & 3);
    e.y = ix(a, e.y, a.nV, site);
    e.z = ix(a, e.z, a.nV, site);
    e.w = ix(a, e.w, a.nV, site);
#else
    (void)a; (void)site;
#endif
    return e;
}
#define IX_INC(a, e) ix_inc((a), (e), __LINE__)

// Launches a kernel; while profiling, the dispatch itself stamps a start and
// an end event (hipExtLaunchKernelGGL), so the recorded duration is the
// kernel's own execution time.
template <typename Kern, typename... Args>
static void launch(jgs2_solver* s, int kid, Kern kernel, dim3 grid, dim3 block, Args... args) {
    if (s->prof) {
        hipEvent_t e0 = pool_event(s), e1 = pool_event(s);
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s->stream, e0, e1, 0, args...);
        s->kt_pending.push_back(jgs2_solver::Pending{kid, e0, e1});
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s->stream, args...);
    }
}

__device__ __forceinline__ int xcd_remap(int i, int nb) {
    const int x = i & 7, j = i >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + j;
}

// v from another lane of the same 16-lane row (DPP move; every lane of a
// wave is active where these are called).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the W lanes of one vertex sub-problem; every lane of the group
// ends with the same total.  Within a row the partners come from DPP moves
// (lane ^ 1, lane ^ 2, then the mirrored lane in the 8- and 16-lane halves,
// each pairing two partial sums that are already equal across their lanes);
// only the step across 16-lane rows goes through ds_bpermute.
template <int W>
__device__ __forceinline__ float lane_sum_w(float v) {
    static_assert(W == 4 || W == 8 || W == 16 || W == 32, "lanes per vertex");
    v += dpp_mov<0xB1>(v);                         // quad_perm(1, 0, 3, 2)
    v += dpp_mov<0x4E>(v);                         // quad_perm(2, 3, 0, 1)
    if constexpr (W >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror
    if constexpr (W >= 16) v += dpp_mov<0x140>(v); // row_mirror
    if constexpr (W >= 32) v += __shfl_xor(v, 16, 32);
    return v;
}

__device__ __forceinline__ float lane_sum(float v) { return lane_sum_w<LPV>(v); }

// Whether free vertex f belongs to a body that is still iterating.
__device__ __forceinline__ bool body_on(const SweepArgs& a, int f) {
    return a.body_on == nullptr || a.body_on[a.fbody[f]] != 0;
}

struct Tet {
    int id[4];
    float D[9];
    float vol, vmu, vlam, mi;
};

__device__ __forceinline__ void load_tet(const float4* __restrict__ tet, int t, Tet& T) {
    const float4* r = tet + (size_t)t * TET_F4;
    const float4 a = r[0], b = r[1], c = r[2], d = r[3], e = r[4];
    T.id[0] = __float_as_int(a.x); T.id[1] = __float_as_int(a.y);
    T.id[2] = __float_as_int(a.z); T.id[3] = __float_as_int(a.w);
    T.D[0] = b.x; T.D[1] = b.y; T.D[2] = b.z; T.D[3] = b.w;
    T.D[4] = c.x; T.D[5] = c.y; T.D[6] = c.z; T.D[7] = c.w;
    T.D[8] = d.x; T.vol = d.y; T.vmu = d.z; T.vlam = d.w; T.mi = e.x;
}

// Tet record without its id word, with the corner ids taken from an
// incidence entry (own corner c is vertex v): the record and the corner
// positions can then be fetched together.
__device__ __forceinline__ void load_tet_inc(const float4* __restrict__ tet, int4 e, int v, Tet& T) {
    const float4* r = tet + (size_t)(e.x >> 2) * TET_F4;
    const float4 b = r[1], c = r[2], d = r[3], f = r[4];
    const int c0 = e.x & 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = (k - c0) & 3;
        int id = v;
        id = q == 1 ? e.y : id;
        id = q == 2 ? e.z : id;
        id = q == 3 ? e.w : id;
        T.id[k] = id;
    }
    T.D[0] = b.x; T.D[1] = b.y; T.D[2] = b.z; T.D[3] = b.w;
    T.D[4] = c.x; T.D[5] = c.y; T.D[6] = c.z; T.D[7] = c.w;
    T.D[8] = d.x; T.vol = d.y; T.vmu = d.z; T.vlam = d.w; T.mi = f.x;
}

// grad N of corner c: rows of Dm^-1 for corners 1..3, minus their sum for 0.
// (Static selects: indexing D with a runtime corner would move the record
// to scratch memory.)
__device__ __forceinline__ void gradN(const float* D, int c, float* gn) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float r0 = D[j], r1 = D[3 + j], r2 = D[6 + j];
        gn[j] = c == 0 ? -(r0 + r1 + r2) : (c == 1 ? r0 : (c == 2 ? r1 : r2));
    }
}

// H = F - I = [u1-u0, u2-u0, u3-u0] Dm^-1 (displacement gradient); the edge
// differences of FP64 displacements are taken in FP64, then rounded
__device__ __forceinline__ void dispgrad(const d4* __restrict__ u, const Tet& T, float* H) {
    const d4 u0 = u[T.id[0]], u1 = u[T.id[1]], u2 = u[T.id[2]], u3 = u[T.id[3]];
    const float du[3][3] = {{(float)(u1.x - u0.x), (float)(u1.y - u0.y), (float)(u1.z - u0.z)},
                            {(float)(u2.x - u0.x), (float)(u2.y - u0.y), (float)(u2.z - u0.z)},
                            {(float)(u3.x - u0.x), (float)(u3.y - u0.y), (float)(u3.z - u0.z)}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            H[3 * i + j] = du[0][i] * T.D[j] + du[1][i] * T.D[3 + j] + du[2][i] * T.D[6 + j];
}

// The same for an FP32 field (the adjoint's y).
__device__ __forceinline__ void dispgrad(const float4* __restrict__ u, const Tet& T, float* H) {
    const float4 u0 = u[T.id[0]], u1 = u[T.id[1]], u2 = u[T.id[2]], u3 = u[T.id[3]];
    const float du[3][3] = {{u1.x - u0.x, u1.y - u0.y, u1.z - u0.z},
                            {u2.x - u0.x, u2.y - u0.y, u2.z - u0.z},
                            {u3.x - u0.x, u3.y - u0.y, u3.z - u0.z}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            H[3 * i + j] = du[0][i] * T.D[j] + du[1][i] * T.D[3 + j] + du[2][i] * T.D[6 + j];
}

__device__ __forceinline__ void load_rot(const float4* __restrict__ R, int v, float* M) {
    const float4 q = R[v];
    rot_from_quat(q.x, q.y, q.z, q.w, M);
}

// Adds w * (U_e^T H_e U_e) for the 12x3 basis U_e whose 3x3 row blocks are
// Phi[b] (b = tet corner): three stress differentials dP[dF_d] with
// dF_d = sum_b Phi_b[:, d] (grad N_b)^T, contracted with dF_e, plus the
// element's inertia share mi * sum_b Phi_b^T Phi_b.
__device__ __forceinline__ void galerkin_hessian(const Tet& T, const Kin<float>& K,
                                                 const float (*Phi)[9], float w, float* A6) {
    float gn[4][3];
#pragma unroll
    for (int b = 0; b < 4; ++b) gradN(T.D, b, gn[b]);
    float dF[3][9];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dF[d][3 * i + j] = Phi[0][3 * i + d] * gn[0][j] + Phi[1][3 * i + d] * gn[1][j] +
                                   Phi[2][3 * i + d] * gn[2][j] + Phi[3][3 * i + d] * gn[3][j];
    int k = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float dP[9];
        snh_dstress(K.F, K.C, 1.0f + K.Jm1, T.vmu, T.vlam, dF[d], dP);
#pragma unroll
        for (int e = d; e < 3; ++e) {
            float s = 0.0f, m = 0.0f;
#pragma unroll
            for (int q = 0; q < 9; ++q) s += dP[q] * dF[e][q];
#pragma unroll
            for (int b = 0; b < 4; ++b)
                m += Phi[b][d] * Phi[b][e] + Phi[b][3 + d] * Phi[b][3 + e] + Phi[b][6 + d] * Phi[b][6 + e];
            A6[k++] += w * (s + T.mi * m);
        }
    }
}

// IPC plane barriers of vertex v at displacement uv: gradient into g and,
// if H6 is given, the Hessian kappa B'' n n^T into H6.
__device__ __forceinline__ void barrier_terms(const SweepArgs& a, int v, const d4& uv, float* g, float* H6) {
    if (a.n_planes == 0) return;
    const float4 X = a.X[v];
    const float x0 = (float)(X.x + uv.x), x1 = (float)(X.y + uv.y), x2 = (float)(X.z + uv.z);
#pragma unroll
    for (int p = 0; p < JGS2_MAX_PLANES; ++p) {
        if (p >= a.n_planes) break;
        const float n0 = a.planes[p][0], n1 = a.planes[p][1], n2 = a.planes[p][2];
        const float d = n0 * x0 + n1 * x1 + n2 * x2 - a.planes[p][3];
        if (d < a.d_hat && d > 0.0f) {
            const float b1 = a.kappa * barrier_d1(d, a.d_hat);
            g[0] += b1 * n0; g[1] += b1 * n1; g[2] += b1 * n2;
            if (H6) {
                const float b2 = a.kappa * barrier_d2(d, a.d_hat);
                H6[0] += b2 * n0 * n0; H6[1] += b2 * n0 * n1; H6[2] += b2 * n0 * n2;
                H6[3] += b2 * n1 * n1; H6[4] += b2 * n1 * n2; H6[5] += b2 * n2 * n2;
            }
        }
    }
}

// Per-vertex feasibility clamp against the static planes: the move is scaled
// by alpha = min(1, 0.9 min_p d_p / (-n_p . step)) over planes it approaches,
// so no vertex reaches a plane whatever the other vertices do.
__device__ __forceinline__ void clamp_step(const SweepArgs& a, int v, const d4& uv, float* step) {
    if (a.n_planes == 0) return;
    const float4 X = a.X[v];
    const float x0 = (float)(X.x + uv.x), x1 = (float)(X.y + uv.y), x2 = (float)(X.z + uv.z);
    float alpha = 1.0f;
#pragma unroll
    for (int p = 0; p < JGS2_MAX_PLANES; ++p) {
        if (p >= a.n_planes) break;
        const float n0 = a.planes[p][0], n1 = a.planes[p][1], n2 = a.planes[p][2];
        const float d = n0 * x0 + n1 * x1 + n2 * x2 - a.planes[p][3];
        const float nd = n0 * step[0] + n1 * step[1] + n2 * step[2];
        if (nd < 0.0f) alpha = fminf(alpha, fmaxf(0.0f, 0.9f * d / (-nd)));
    }
    step[0] *= alpha; step[1] *= alpha; step[2] *= alpha;
}

template <int NV, int W>
__device__ __forceinline__ void block_partial_t(double val, bool lane0, double* partial) {
    __shared__ double sp[NV];
    const int vloc = threadIdx.x / W;
    if (lane0) sp[vloc] = val;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < NV; ++i) s += sp[i];
        partial[blockIdx.x] = s;
    }
}

__device__ __forceinline__ void block_partial(double val, bool lane0, double* partial) {
    block_partial_t<VPB, LPV>(val, lane0, partial);
}

// ---------------------------------------------------------------------------
// Phase 1: assembled gradient g_a (elastic + inertia + barrier), the
// volume-weighted mean deformation gradient of the incident tets and its
// polar rotation R_a; per-block partial sums of |g|^2 (FP64).
// ---------------------------------------------------------------------------
// One incident tet's share of g_v and of the volume-weighted F sum, added
// with weight w (own corner e.x & 3 is vertex v).  The gradient is evaluated
// in FP64 (displacement gradient from the FP64 positions, stress and sum):
// its terms (elastic, inertial, external) nearly cancel at a converged step,
// so an FP32 evaluation would floor the relative residual of stiff bodies
// near 1e-4.  The rotation's F sum stays FP32.
__device__ __forceinline__ void phase1_term(const SweepArgs& a, const int4 e, int v, double w, double* g,
                                            float* Fs) {
    const int c = e.x & 3;
    Tet T;
    load_tet_inc(a.tet, IX_INC(a, e), v, T);
    const d4 u0 = a.u[T.id[0]], u1 = a.u[T.id[1]], u2 = a.u[T.id[2]], u3 = a.u[T.id[3]];
    const double du[3][3] = {{u1.x - u0.x, u1.y - u0.y, u1.z - u0.z},
                             {u2.x - u0.x, u2.y - u0.y, u2.z - u0.z},
                             {u3.x - u0.x, u3.y - u0.y, u3.z - u0.z}};
    double D[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) D[i] = (double)T.D[i];
    double H[9], cH[9], P[9], gn[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) H[3 * i + j] = du[0][i] * D[j] + du[1][i] * D[3 + j] + du[2][i] * D[6 + j];
    Kin<double> K;
    kinematics(H, K, cH);
    snh_stress_H(H, K, cH, (double)T.vmu, (double)T.vlam, P);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double r0 = D[j], r1 = D[3 + j], r2 = D[6 + j];
        gn[j] = c == 0 ? -(r0 + r1 + r2) : (c == 1 ? r0 : (c == 2 ? r1 : r2));
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = fma(w, P[3 * i] * gn[0] + P[3 * i + 1] * gn[1] + P[3 * i + 2] * gn[2], g[i]);
    const float wv = (float)w * T.vol;
#pragma unroll
    for (int i = 0; i < 9; ++i) Fs[i] = fmaf(wv, (float)K.F[i], Fs[i]);
}

__device__ __forceinline__ double lane_sum_d(double v) {
#pragma unroll
    for (int o = LPV / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPV);
    return v;
}

// GATED (several bodies, inside a step's sweeps): rows of bodies that have
// stopped are skipped before any gather; their g and R are those of their
// frozen positions already.  Otherwise every lane gathers its first incident
// tet unconditionally.
template <bool GATED>
__global__ __launch_bounds__(BLOCK) void k_phase1(SweepArgs a, int want_R) {
    const int lane = threadIdx.x % LPV;
    const int vloc = threadIdx.x / LPV;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int idx = blk * VPB + vloc;
    const int nidx = a.list ? a.n_list : a.nVf;
    const bool in_range = idx < nidx;
    const int f = in_range ? (a.list ? IX(a, a.list[idx], a.nVf) : idx) : 0;
    const bool active = GATED ? (in_range && a.body_on[a.fbody[f]] != 0) : in_range;
    // Row-level loads first and without branches (f is a valid row even out
    // of range; rows are padded to maxi entries); every lane then gathers its
    // first incident tet before n is tested (padding reads tet 0 and vertex 0
    // and adds with weight 0), so a lane waits on row -> corners -> positions.
    const int v = IX(a, a.free_ids[f], a.nV);
    const int n = a.inc_n[f];
    const int4 e0 = GATED ? make_int4(0, 0, 0, 0) : a.inc4[(size_t)f * a.maxi + min(lane, a.maxi - 1)];
    const d4 uv = a.u[v], zv = a.zu[v];
    double g[3] = {0.0, 0.0, 0.0};
    float Fs[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int j0 = lane;
    if constexpr (!GATED) {
        const bool has = lane < n;
        const int4 e = make_int4(has ? e0.x : 0, has ? e0.y : 0, has ? e0.z : 0, has ? e0.w : 0);
        phase1_term(a, e, v, has ? 1.0 : 0.0, g, Fs);
        j0 += LPV;
    }
    if (active)
        for (int j = j0; j < n; j += LPV) phase1_term(a, a.inc4[(size_t)f * a.maxi + j], v, 1.0, g, Fs);
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = lane_sum_d(g[i]);
    if (want_R) {
#pragma unroll
        for (int i = 0; i < 9; ++i) Fs[i] = lane_sum(Fs[i]);
    }
    double gsq = 0.0;
    if (active && lane == 0) {
        const double m = zv.w;
        g[0] += m * (uv.x - zv.x);
        g[1] += m * (uv.y - zv.y);
        g[2] += m * (uv.z - zv.z);
        float gb[3] = {0.f, 0.f, 0.f};
        barrier_terms(a, v, uv, gb, nullptr);
        g[0] += gb[0]; g[1] += gb[1]; g[2] += gb[2];
        a.g[v] = make_float4((float)g[0], (float)g[1], (float)g[2], 0.0f);
        gsq = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (want_R) {
            float mx = 0.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) mx = fmaxf(mx, fabsf(Fs[i]));
            const float inv = mx > 0.0f ? 1.0f / mx : 1.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) Fs[i] *= inv;
            float R[9], q[4];
            polar_rotation(Fs, R);
            quat_from_rot(R, q);
            a.R[v] = make_float4(q[0], q[1], q[2], q[3]);
        }
    }
    block_partial(gsq, active && lane == 0, a.partial);
}

// ---------------------------------------------------------------------------
// Phase 2, cubature variant (reading R3 of the correction):
//   A_i = sum_{e ni i} U_e^T H_e U_e + H^B_i + sum_s w_s U_s^T H_s U_s
//   b_i = g_i + sum_{a in N(i)} Phi_{i,a}^T g_a
//         + sum_s sum_{a in s, a not in Nbar(i)} (w_s / n_a) Phi_{i,a}^T g_a
// with Phi_{i,a} = R_a Ubar_{i,a} R_i^T (Eq. tilde_phi); then
// x_i <- x_i - omega A_i^-1 b_i (Eq. reduced_local).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void corotate(const float* U, const float* Ri, const float* Ra, float* Phi) {
    float T9[9];  // U R_i^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T9[3 * i + j] = U[3 * i] * Ri[3 * j] + U[3 * i + 1] * Ri[3 * j + 1] + U[3 * i + 2] * Ri[3 * j + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Phi[3 * i + j] = Ra[3 * i] * T9[j] + Ra[3 * i + 1] * T9[3 + j] + Ra[3 * i + 2] * T9[6 + j];
}

__global__ __launch_bounds__(BLOCK) void k_phase2_cubature(SweepArgs a) {
    __shared__ float sPhi[VPB][KMAX][9];
    const int lane = threadIdx.x % LPV;
    const int vloc = threadIdx.x / LPV;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int idx = blk * VPB + vloc;
    const int nidx = a.list ? a.n_list : a.nVf;
    const bool in_range = idx < nidx;
    const int f = in_range ? (a.list ? a.list[idx] : idx) : 0;
    const bool active = in_range && body_on(a, f);
    const int v = a.free_ids[f];
    if (in_range && !active && lane == 0) a.unext[v] = a.u[v];  // converged body: unchanged
    float Ri[9];
    load_rot(a.R, v, Ri);
    float A6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, b[3] = {0.f, 0.f, 0.f};

    // one-ring rows: Phi_{i,a} into LDS, gradient projection
    const int nr = active ? a.ring_n[f] : 0;
    for (int k = lane; k < nr; k += LPV) {
        const int av = a.ring[(size_t)f * a.K + k];
        float U[9], Ra[9], Phi[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) U[q] = a.Uring[((size_t)f * 9 + q) * a.K + k];
        load_rot(a.R, av, Ra);
        corotate(U, Ri, Ra, Phi);
#pragma unroll
        for (int q = 0; q < 9; ++q) sPhi[vloc][k][q] = Phi[q];
        const float4 ga = a.g[av];
#pragma unroll
        for (int j = 0; j < 3; ++j) b[j] += Phi[j] * ga.x + Phi[3 + j] * ga.y + Phi[6 + j] * ga.z;
    }
    __syncthreads();

    // incident tets, exact Galerkin blocks
    const int ni = active ? a.inc_n[f] : 0;
    for (int j = lane; j < ni; j += LPV) {
        const int pk = a.inc[(size_t)f * a.maxi + j];
        const uint32_t sl = a.incslot[(size_t)f * a.maxi + j];
        Tet T;
        load_tet(a.tet, pk >> 2, T);
        float H[9], cH[9];
        Kin<float> K;
        dispgrad(a.u, T, H);
        kinematics(H, K, cH);
        float Phi[4][9];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint32_t s = (sl >> (8 * c)) & 0xFFu;
            if (s == SLOT_SELF) {
#pragma unroll
                for (int q = 0; q < 9; ++q) Phi[c][q] = (q % 4 == 0) ? 1.0f : 0.0f;
            } else if (s == SLOT_NONE) {
#pragma unroll
                for (int q = 0; q < 9; ++q) Phi[c][q] = 0.0f;
            } else {
#pragma unroll
                for (int q = 0; q < 9; ++q) Phi[c][q] = sPhi[vloc][s][q];
            }
        }
        galerkin_hessian(T, K, Phi, 1.0f, A6);
    }

    // cubature samples on the last S lanes
    const int s = lane - (LPV - a.S);
    if (active && s >= 0) {
        const int e = a.samp_e[(size_t)f * a.S + s];
        if (e >= 0) {
            const float* rec = a.samp + (size_t)f * SREC * a.S;
            const float w = rec[s];
            Tet T;
            load_tet(a.tet, e, T);
            float H[9], cH[9];
            Kin<float> K;
            dispgrad(a.u, T, H);
            kinematics(H, K, cH);
            float Phi[4][9];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int av = T.id[c];
                float U[9], Ra[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) U[q] = rec[(5 + 9 * c + q) * a.S + s];
                load_rot(a.R, av, Ra);
                corotate(U, Ri, Ra, Phi[c]);
                const float gc = rec[(1 + c) * a.S + s];
                if (gc != 0.0f) {
                    const float4 ga = a.g[av];
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj)
                        b[jj] += gc * (Phi[c][jj] * ga.x + Phi[c][3 + jj] * ga.y + Phi[c][6 + jj] * ga.z);
                }
            }
            galerkin_hessian(T, K, Phi, w, A6);
        }
    }

#pragma unroll
    for (int i = 0; i < 6; ++i) A6[i] = lane_sum(A6[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = lane_sum(b[i]);
    if (active && lane == 0) {
        const d4 uv = a.u[v];
        float gv[3] = {0.f, 0.f, 0.f};
        barrier_terms(a, v, uv, gv, A6);  // barrier Hessian of vertex i only (g already holds its gradient)
        float A[9] = {A6[0], A6[1], A6[2], A6[1], A6[3], A6[4], A6[2], A6[4], A6[5]};
        const float4 gi = a.g[v];
        const float bb[3] = {b[0] + gi.x, b[1] + gi.y, b[2] + gi.z};
        float dx[3];
        local_solve(A, bb, dx);
        float st[3] = {a.omega * dx[0], a.omega * dx[1], a.omega * dx[2]};
        clamp_step(a, v, uv, st);
        a.unext[v] = make_d4(uv.x + st[0], uv.y + st[1], uv.z + st[2], 0.0);
    }
}

// ---------------------------------------------------------------------------
// Plain per-vertex Newton relaxation, A_i = H_ii, fused in one pass; in the
// residual-only mode (no_write) it leaves per-block |b|^2 partials of the
// iterate it read instead of updating it.
// LIN = false: b_i = g_i, x_i <- x_i - omega H_ii^-1 g_i (forward sweep).
// LIN = true : b_i = (H y - rhs)_i with H the Hessian at u (held fixed): a
//              linear sweep on H y = rhs for the adjoint; the incident
//              tets contribute dP[dF(y)] grad N, the vertex m/h^2 y and the
//              barrier Hessian times y.
// W lanes share a vertex (each takes every W-th incident tet), BLK threads
// per block hold BLK / W vertices: the launch shapes the tuner chooses from.
// ---------------------------------------------------------------------------
// Terms of one incidence (tet T, own corner c) for the plain and linear
// sweeps, added with weight w (1 or 0: a zero weight keeps the gathers
// unconditional): the element's share of g_v (or of (H y)_v) and of the
// diagonal block H_vv.
// 16-byte load marked non-temporal (streamed data, read once).
__device__ __forceinline__ float4 load_nt(const float4* p) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// Incidence record (planes stride apart): the tet's Dm^-1, V mu, V lam, V and
// corner ids; the own corner c is the corner whose id is the row's vertex
// (zero padding records name vertex 0 and are added with weight 0).
template <bool NT>
__device__ __forceinline__ void load_irec(const float4* __restrict__ r, int stride, int vself, Tet& T, int& c) {
    // each record is read once per sweep; when the records outgrow the
    // last-level cache (NT) they are streamed (non-temporal), which keeps the
    // reused corner positions resident
    float4 p0, p1, p2, p3;
    if constexpr (NT) {
        p0 = load_nt(r); p1 = load_nt(r + stride); p2 = load_nt(r + 2 * stride); p3 = load_nt(r + 3 * stride);
    } else {
        p0 = r[0]; p1 = r[stride]; p2 = r[2 * stride]; p3 = r[3 * stride];
    }
    T.D[0] = p0.x; T.D[1] = p0.y; T.D[2] = p0.z; T.D[3] = p0.w;
    T.D[4] = p1.x; T.D[5] = p1.y; T.D[6] = p1.z; T.D[7] = p1.w;
    T.D[8] = p2.x; T.vmu = p2.y; T.vlam = p2.z; T.vol = p2.w;
    T.id[0] = __float_as_int(p3.x); T.id[1] = __float_as_int(p3.y);
    T.id[2] = __float_as_int(p3.z); T.id[3] = __float_as_int(p3.w);
    c = T.id[0] == vself ? 0 : (T.id[1] == vself ? 1 : (T.id[2] == vself ? 2 : 3));
    T.mi = 0.0f;
}

// The corner ids of an incidence record, checked (bounds-checked build).
__device__ __forceinline__ void ix_ids(const SweepArgs& a, Tet& T, int site) {
#ifdef JGS2_BOUNDS_CHECK
#pragma unroll
    for (int k = 0; k < 4; ++k) T.id[k] = ix(a, T.id[k], a.nV, site);
#else
    (void)a; (void)T; (void)site;
#endif
}
#define IX_IDS(a, T) ix_ids((a), (T), __LINE__)

template <bool LIN>
__device__ __forceinline__ void plain_tet_term(const SweepArgs& a, const Tet& T, int c, float w, float* g, float* A6) {
    float H[9], cH[9], gn[3], t[3];
    Kin<float> K;
    dispgrad(a.u, T, H);
    kinematics(H, K, cH);
    gradN(T.D, c, gn);
    if (LIN) {
        float dY[9], dP[9];
        dispgrad(a.ly, T, dY);
        snh_dstress(K.F, K.C, 1.0f + K.Jm1, T.vmu, T.vlam, dY, dP);
#pragma unroll
        for (int i = 0; i < 3; ++i) t[i] = dP[3 * i] * gn[0] + dP[3 * i + 1] * gn[1] + dP[3 * i + 2] * gn[2];
    } else {
        float P[9];
        snh_stress_H(H, K, cH, T.vmu, T.vlam, P);
#pragma unroll
        for (int i = 0; i < 3; ++i) t[i] = P[3 * i] * gn[0] + P[3 * i + 1] * gn[1] + P[3 * i + 2] * gn[2];
    }
    // own diagonal block: dP[e_d gn^T] : e_e gn^T.  The cofactor-derivative
    // term is (e_e x e_d)^T F (gn x gn) = 0 here, leaving
    // V mu |gn|^2 I + V lam (cof F gn)(cof F gn)^T
    const float c0 = K.C[0] * gn[0] + K.C[1] * gn[1] + K.C[2] * gn[2];
    const float c1 = K.C[3] * gn[0] + K.C[4] * gn[1] + K.C[5] * gn[2];
    const float c2 = K.C[6] * gn[0] + K.C[7] * gn[1] + K.C[8] * gn[2];
    const float mg = T.vmu * (gn[0] * gn[0] + gn[1] * gn[1] + gn[2] * gn[2]);
    const float h[6] = {mg + T.vlam * c0 * c0, T.vlam * c0 * c1, T.vlam * c0 * c2,
                        mg + T.vlam * c1 * c1, T.vlam * c1 * c2, mg + T.vlam * c2 * c2};
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = fmaf(w, t[i], g[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) A6[i] = fmaf(w, h[i], A6[i]);
}

// One cubature sample's damper term, spread over the four lanes of a quad
// (lane b of the quad takes tet corner b): each lane co-rotates its corner's
// U-bar row, Phi_b = R_b U-bar_{i,b} R_i^T, and forms its share of the three
// directional deformation-gradient differentials dF_d = sum_b Phi_b[:, d]
// (grad N_b)^T and of the inertia product sum_b Phi_b^T Phi_b; quad sums
// complete them, then lane d < 3 evaluates the stress differential dP[dF_d]
// and adds w (dP[dF_d] : dF_e + m_i (Phi^T Phi)_de) for e >= d to A6.  Every
// lane of the quad must be active (the quad sums are DPP moves inside it).
__device__ __forceinline__ float quad_sum(float v) {
    v += dpp_mov<0xB1>(v);  // quad_perm(1, 0, 3, 2)
    v += dpp_mov<0x4E>(v);  // quad_perm(2, 3, 0, 1)
    return v;
}

__device__ __forceinline__ void damper_sample_quad(const SweepArgs& a, int e, int b, const float* rec, int sm,
                                                   const float* Ri, float* A6) {
    Tet T;
    load_tet(a.tet, e, T);
    float H[9], cH[9];
    Kin<float> K;
    dispgrad(a.u, T, H);
    kinematics(H, K, cH);
    const int vb = b == 0 ? T.id[0] : (b == 1 ? T.id[1] : (b == 2 ? T.id[2] : T.id[3]));
    float U[9], Ra[9], Phi[9], gn[3];
#pragma unroll
    for (int qq = 0; qq < 9; ++qq) U[qq] = rec[(5 + 9 * b + qq) * a.S + sm];
    load_rot(a.R, vb, Ra);
    corotate(U, Ri, Ra, Phi);
    gradN(T.D, b, gn);
    float dF[3][9];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) dF[d][3 * i + j] = quad_sum(Phi[3 * i + d] * gn[j]);
    float m6[6];
    {
        int k = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int f = d; f < 3; ++f)
                m6[k++] = quad_sum(Phi[d] * Phi[f] + Phi[3 + d] * Phi[3 + f] + Phi[6 + d] * Phi[6 + f]);
    }
    // lane b < 3 takes direction d = b (lane 3 repeats d = 0 and adds nothing)
    float dFd[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) dFd[q] = b == 1 ? dF[1][q] : (b == 2 ? dF[2][q] : dF[0][q]);
    float dP[9];
    snh_dstress(K.F, K.C, 1.0f + K.Jm1, T.vmu, T.vlam, dFd, dP);
    float s3[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < 9; ++q) acc += dP[q] * dF[f][q];
        s3[f] = acc;
    }
    const float w = rec[sm];
    const float mi = T.mi;
    // A6 = (00, 01, 02, 11, 12, 22); m6 in the same order (selects, so that
    // A6 stays in registers)
    A6[0] += b == 0 ? w * (s3[0] + mi * m6[0]) : 0.0f;
    A6[1] += b == 0 ? w * (s3[1] + mi * m6[1]) : 0.0f;
    A6[2] += b == 0 ? w * (s3[2] + mi * m6[2]) : 0.0f;
    A6[3] += b == 1 ? w * (s3[1] + mi * m6[3]) : 0.0f;
    A6[4] += b == 1 ? w * (s3[2] + mi * m6[4]) : 0.0f;
    A6[5] += b == 2 ? w * (s3[2] + mi * m6[5]) : 0.0f;
}

// DAMP (forward only): the damper reading of the correction fused into the
// same pass, A_i = H_ii + sum_s w_s Phi_s^T H_s Phi_s with Phi_{i,a} =
// R_a Ubar_{i,a} R_i^T over the row's cubature samples, b_i = g_i; each
// sample goes to one quad of the row's lanes (W / 4 samples per round),
// rotations are those of the last rotation (or phase-1) pass.
// Rows blk * NV .. blk * NV + NV - 1 of the range [cbase, cbase + nidx) (rows
// in colour order: a colour is a contiguous range, a Jacobi sweep the whole
// range, so no list is read before the rows).
template <bool LIN, int W, int BLK, bool SPEC, bool NT, bool DAMP = false>
__device__ __forceinline__ void plain_body(const SweepArgs& a, int blk, int cbase, int nidx) {
    constexpr int NV = BLK / W;
    const int lane = threadIdx.x % W;
    const int vloc = threadIdx.x / W;
    const int idx = blk * NV + vloc;
    const bool in_range = idx < nidx;
    const int q = in_range ? cbase + idx : 0;
    // Everything that needs only the row index is fetched up front and
    // without branches (q is a valid row even out of range; rows are padded
    // to maxi entries): the row's count, this lane's first incidence record
    // (contiguous across the lanes of a row) and the vertex's own records.
    // SPEC (one body, or a linear sweep): the stop flag is the same for every
    // row, and the first record's corner positions are gathered by every lane
    // before the flag or n is tested (zero records name vertex 0 and add with
    // weight 0), so a lane waits on two levels: records -> positions.
    const int vself = IX(a, a.vid_c[q], a.nV);
    const int n = a.incn_c[q];
    const float4* row = a.irec_c + (size_t)q * IREC_F4 * a.maxi;
    Tet T0, T1;
    int c0 = 0, c1 = 0;
    if constexpr (SPEC) {
        load_irec<NT>(row + min(lane, a.maxi - 1), a.maxi, vself, T0, c0);
        IX_IDS(a, T0);
    }
    if constexpr (SPEC && W < 32) {
        load_irec<NT>(row + min(lane + W, a.maxi - 1), a.maxi, vself, T1, c1);
        IX_IDS(a, T1);
    }
    const d4 uv = a.u[vself];
    d4 zv = make_d4(0.0, 0.0, 0.0, 0.0);
    float4 yv = make_float4(0.f, 0.f, 0.f, 0.f), rv = yv;
    float mlin = 0.f;
    if (LIN) { yv = a.ly[vself]; rv = a.lrhs[vself]; mlin = a.mh2[vself]; }
    else zv = a.zu[vself];
    const int flag = LIN ? 1 : (SPEC ? a.body_on[0] : a.body_on[a.fbody_c[q]]);
    const bool active = in_range & (flag != 0);
    float g[3] = {0.f, 0.f, 0.f}, A6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // Lane l takes entries l, l + W, ... (the order of its partial sums).  The
    // sums of an inactive row are never used, so with SPEC the first entry is
    // added with a weight that needs only n.
    int j0 = lane;
    if constexpr (SPEC) {
        // entries past n are zero records or a repeat of the row's last one
        plain_tet_term<LIN>(a, T0, c0, lane < n ? 1.0f : 0.0f, g, A6);
        j0 += W;
        if constexpr (W < 32) {
            // a second round, also gathered before n or the flag is known
            plain_tet_term<LIN>(a, T1, c1, j0 < n ? 1.0f : 0.0f, g, A6);
            j0 += W;
        }
    }
    if (active)
        for (int j = j0; j < n; j += W) {
            Tet T;
            int c;
            load_irec<NT>(row + j, a.maxi, vself, T, c);
            IX_IDS(a, T);
            plain_tet_term<LIN>(a, T, c, 1.0f, g, A6);
        }
    if constexpr (DAMP && !LIN) {
        constexpr int SPR = W / 4;  // samples per round, one quad of lanes each
        if (active) {
            const int f = a.free_c[q];
            const float* rec = a.samp + (size_t)f * SREC * a.S;
            float Ri[9];
            load_rot(a.R, vself, Ri);
            const int qd = lane >> 2, b = lane & 3;
            for (int sm0 = 0; sm0 < a.S; sm0 += SPR) {
                const int sm = sm0 + qd;
                const int e = sm < a.S ? a.samp_e[(size_t)f * a.S + sm] : -1;
                if (e >= 0) damper_sample_quad(a, e, b, rec, sm, Ri, A6);  // the quad's lanes agree on e
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = lane_sum_w<W>(g[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) A6[i] = lane_sum_w<W>(A6[i]);
    if (!LIN && in_range && !active && lane == 0 && !a.in_place)
        a.unext[vself] = uv;  // converged body in a Jacobi sweep: carried over unchanged
    double gsq = 0.0;
    if (active && lane == 0) {
        const int v = vself;
        if (LIN) {
            const float m = mlin;
            float Hb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, gb[3] = {0.f, 0.f, 0.f};
            barrier_terms(a, v, uv, gb, Hb);
            g[0] += m * yv.x - rv.x + Hb[0] * yv.x + Hb[1] * yv.y + Hb[2] * yv.z;
            g[1] += m * yv.y - rv.y + Hb[1] * yv.x + Hb[3] * yv.y + Hb[4] * yv.z;
            g[2] += m * yv.z - rv.z + Hb[2] * yv.x + Hb[4] * yv.y + Hb[5] * yv.z;
            A6[0] += m + Hb[0]; A6[1] += Hb[1]; A6[2] += Hb[2];
            A6[3] += m + Hb[3]; A6[4] += Hb[4]; A6[5] += m + Hb[5];
        } else {
            const float m = (float)zv.w;
            g[0] += m * (float)(uv.x - zv.x);
            g[1] += m * (float)(uv.y - zv.y);
            g[2] += m * (float)(uv.z - zv.z);
            A6[0] += m; A6[3] += m; A6[5] += m;
            barrier_terms(a, v, uv, g, A6);
        }
        gsq = (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
        if (LIN && a.lres) a.lres[v] = make_float4(g[0], g[1], g[2], 0.0f);
        if (!a.no_write) {
            float A[9] = {A6[0], A6[1], A6[2], A6[1], A6[3], A6[4], A6[2], A6[4], A6[5]};
            float dx[3];
            local_solve(A, g, dx);
            float st[3] = {a.omega * dx[0], a.omega * dx[1], a.omega * dx[2]};
            if (LIN) {
                float4* out = a.in_place ? const_cast<float4*>(a.ly) : a.lynext;
                out[v] = make_float4(yv.x + st[0], yv.y + st[1], yv.z + st[2], 0.0f);
            } else {
                clamp_step(a, v, uv, st);
                d4* out = a.in_place ? const_cast<d4*>(a.u) : a.unext;
                out[v] = make_d4(uv.x + st[0], uv.y + st[1], uv.z + st[2], 0.0);
            }
        }
    }
    if (a.no_write) block_partial_t<NV, W>(gsq, active && lane == 0, a.partial);  // uniform branch
}

#define PLAIN_ROWS(a) xcd_remap(blockIdx.x, gridDim.x), (a).cbase, (a).list ? (a).n_list : (a).nVf
template <int W, int BLK, bool SPEC, bool NT>
__global__ __launch_bounds__(BLK) void k_plain(SweepArgs a) { plain_body<false, W, BLK, SPEC, NT>(a, PLAIN_ROWS(a)); }
template <int W, int BLK, bool SPEC, bool NT>
__global__ __launch_bounds__(BLK) void k_damper(SweepArgs a) {
    plain_body<false, W, BLK, SPEC, NT, true>(a, PLAIN_ROWS(a));
}
template <int W, int BLK, bool NT>
__global__ __launch_bounds__(BLK) void k_linear(SweepArgs a) { plain_body<true, W, BLK, true, NT>(a, PLAIN_ROWS(a)); }
#undef PLAIN_ROWS

// A whole group of k coloured Gauss-Seidel sweeps (plain variant, forward) in
// one cooperative launch: every block walks the row blocks of colour c
// (block b takes b, b + gridDim, ...), then the grid waits at a barrier
// before colour c + 1; before the group's last sweep the grid keeps the
// iterate for the |dx| check.  The launch holds no more blocks than the
// device keeps resident at once (the runtime refuses a larger cooperative
// launch), and every block reaches every barrier: the loops are uniform and
// plain_body has no early exit.  The same rows see the same arithmetic as in
// one launch per colour, so the result is bitwise that of those launches.
template <int W, int BLK, bool SPEC, bool NT>
__global__ __launch_bounds__(BLK) void k_plain_persistent(SweepArgs a, int k, const int* __restrict__ col_off,
                                                           int n_colors, d4* __restrict__ uprev) {
    constexpr int NV = BLK / W;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    // blocks are dealt to the 8 XCDs in turn (block i on XCD i % 8): each XCD's
    // blocks take a contiguous eighth of a colour's row blocks, as xcd_remap
    // gives a one-launch-per-colour grid (the grid is a multiple of 8)
    const int xcd = blockIdx.x & 7, rank = blockIdx.x >> 3, per = gridDim.x >> 3;
    for (int it = 0; it < k; ++it) {
        if (it == k - 1) {
            for (int i = blockIdx.x * BLK + threadIdx.x; i < a.nV; i += gridDim.x * BLK) uprev[i] = a.u[i];
            grid.sync();
        }
        for (int c = 0; c < n_colors; ++c) {
            const int c0 = col_off[c], n = col_off[c + 1] - c0;
            const int nb = (n + NV - 1) / NV;
            const int q = nb >> 3, r = nb & 7;
            const int lo = xcd * q + min(xcd, r), hi = lo + q + (xcd < r ? 1 : 0);
            for (int b = lo + rank; b < hi; b += per) plain_body<false, W, BLK, SPEC, NT>(a, b, c0, n);
            grid.sync();
        }
    }
}

// Per-vertex rotations alone (Sec. 4.3): R_a is the polar rotation of the
// volume-weighted mean deformation gradient of a's incident tets, the same
// quantity as in phase 1, gathered from the colour-ordered incidence records.
// The damper sweeps need only these.  Rows of a stopped body (several
// bodies) keep their rotations.  W lanes gather each row's records; the
// block's NV = BLK / W summed gradients then go through LDS so that NV
// threads of the first wave run one polar decomposition each (with W = 8,
// BLK = 512 that is 64 decompositions side by side per wave).
template <int W, int BLK, bool SPEC, bool NT>
__global__ __launch_bounds__(BLK) void k_rot(SweepArgs a) {
    constexpr int NV = BLK / W;
    static_assert(NV <= 64, "one wave runs the block's decompositions");
    __shared__ float sF[NV][9];
    __shared__ int sV[NV];
    const int lane = threadIdx.x % W;
    const int vloc = threadIdx.x / W;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int idx = blk * NV + vloc;
    const bool in_range = idx < a.nVf;
    const int q = in_range ? idx : 0;
    const int vself = IX(a, a.vid_c[q], a.nV);
    const int n = a.incn_c[q];
    const float4* row = a.irec_c + (size_t)q * IREC_F4 * a.maxi;
    // the first record of every lane is gathered before n or the body flag
    // is tested (added with weight 0 where unused)
    Tet T0;
    int c0 = 0;
    load_irec<NT>(row + min(lane, a.maxi - 1), a.maxi, vself, T0, c0);
    IX_IDS(a, T0);
    const int flag = SPEC ? a.body_on[0] : a.body_on[a.fbody_c[q]];
    const bool active = in_range & (flag != 0);
    // sums of V_e (F_e - I) and of V_e over the incident tets
    float Hs[9], vs;
    {
        float H[9];
        dispgrad(a.u, T0, H);
        const float w = lane < n ? T0.vol : 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) Hs[i] = w * H[i];
        vs = w;
    }
    if (active)
        for (int j = lane + W; j < n; j += W) {
            Tet T;
            int c;
            load_irec<NT>(row + j, a.maxi, vself, T, c);
            IX_IDS(a, T);
            float H[9];
            dispgrad(a.u, T, H);
#pragma unroll
            for (int i = 0; i < 9; ++i) Hs[i] = fmaf(T.vol, H[i], Hs[i]);
            vs += T.vol;
        }
#pragma unroll
    for (int i = 0; i < 9; ++i) Hs[i] = lane_sum_w<W>(Hs[i]);
    vs = lane_sum_w<W>(vs);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) sF[vloc][i] = Hs[i] + ((i % 4 == 0) ? vs : 0.0f);
        sV[vloc] = active ? vself : -1;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = sV[threadIdx.x];
        if (v >= 0) {
            float Fs[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) Fs[i] = sF[threadIdx.x][i];
            float mx = 0.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) mx = fmaxf(mx, fabsf(Fs[i]));
            const float inv = mx > 0.0f ? 1.0f / mx : 1.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) Fs[i] *= inv;
            float R[9], qv[4];
            polar_rotation(Fs, R);
            quat_from_rot(R, qv);
            a.R[v] = make_float4(qv[0], qv[1], qv[2], qv[3]);
        }
    }
}

// ---------------------------------------------------------------------------
// Exact co-rotated subspace (the literal form of Eq. local_newton with the
// derivatives of Eq. relation and the co-rotated rows of Eq. tilde_phi):
//   b_f = sum_a Phi_{f,a}^T g_a = R_f B_f^-1 (H-bar^-1 h)_f,  h_a = R_a^T g_a
// (U-bar_{f,a} = (H-bar^-1)_{a,f} B_f^-1 by Eq. u, and H-bar^-1 is symmetric),
//   A_f = m_f / h^2 I + H^B_f + sum_{e ni f} sum_b H_e[c_f, b] Phi_{f,b}
// with Phi_{f,b} = R_b U-bar_{f,b} R_f^T (the identity at b = f, zero at pinned
// b), A_f symmetrised, x_f <- x_f - omega A_f^-1 b_f.  H-bar^-1 is kept once,
// as the lower triangle of 64 x 64-vertex tiles over the positions q.
// ---------------------------------------------------------------------------
constexpr size_t MT_TILE = (size_t)MT_Q * 9 * MT_Q;  // floats per tile

__device__ __forceinline__ size_t tile_index(int I, int J) { return (size_t)I * (I + 1) / 2 + J; }

// Rest-frame gradients h_q = R_a^T g_a in position order.
__global__ __launch_bounds__(256) void k_hvec(SweepArgs a) {
    const int qx = blockIdx.x * blockDim.x + threadIdx.x;
    if (qx >= a.nVf) return;
    const int v = IX(a, a.qvert[qx], a.nV);
    const float4 g = a.g[v];
    float R[9];
    load_rot(a.R, v, R);
    a.hvec[qx] = make_float4(R[0] * g.x + R[3] * g.y + R[6] * g.z, R[1] * g.x + R[4] * g.y + R[7] * g.z,
                             R[2] * g.x + R[5] * g.y + R[8] * g.z, 0.0f);
}

// y = H-bar^-1 h over super-tiles of MT_SG x MT_SG tiles: block (SI, SJ),
// SI >= SJ, of MT_SG waves; wave w takes tile row I = MT_SG SI + w across the
// stored tiles (I, J) of tile columns J = MT_SG SJ .. MT_SG SJ + MT_SG - 1,
// J <= I.  Lane (s, c) = (lane / 16, lane % 16) reads columns 4c .. 4c + 3 of
// rows il = 4k + s as 16-byte loads, two 4-row batches (18 loads) in flight;
// the zero-filled padding past nVf (of the tiles and of h) reads as zero and
// batches wholly past it are skipped.  Each tile is read once,
// non-temporally, and applied both ways:
//  * row parts (M h_J): summed over the row's 16 lanes by DPP and kept by
//    lane (s, k) for row 4k + s, accumulated over the wave's tiles in column
//    order, then stored once per wave as prow[SJ][I];
//  * column parts of off-diagonal tiles (M^T h_I): summed per lane, then over
//    the four 16-lane rows, into LDS; after the block's barrier wave j sums
//    the column parts of tile column MT_SG SJ + j over the waves in order and
//    stores pcol[SI][J].
// Each super-tile thus writes 2 MT_SG partial vectors for MT_SG^2 tiles
// (stores interleaved with the streamed reads cost HBM time in proportion to
// their bytes), as non-temporal stores.  Every sum runs in a fixed order: no
// atomics, the result is bitwise-deterministic.  Indices are wave-uniform and
// kept in scalar registers.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// HALF: the tiles in FP16, each entry stored divided by its tile's scale;
// 8-byte loads, four 4-row batches in flight, products in FP32 from the
// converted entries, the tile's row and column parts multiplied by the scale.
template <bool HALF>
__global__ __launch_bounds__(64 * MT_SG) void k_symv(SweepArgs a) {
    __shared__ float sCol[MT_SG][MT_SG][3][MT_Q];  // [wave][tile column][component][column]
    // a sweep issued after every body stopped (the host reads residuals one
    // group late) changes nothing: skip its stream (uniform over the block)
    if (a.nactive && *a.nactive == 0) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nsq = ((a.nVf + MT_Q - 1) / MT_Q + MT_SG - 1) / MT_SG;  // super-rows
    const int bt = a.slist ? IX(a, a.slist[blockIdx.x], (long long)nsq * (nsq + 1) / 2) : (int)blockIdx.x;
    const uint64_t live = a.smask ? a.smask[bt] : ~0ull;  // bit w MT_SG + j: tile streamed
    // bt = SI (SI + 1) / 2 + SJ, SJ <= SI
    int SI = __builtin_amdgcn_readfirstlane((int)((sqrtf(8.0f * (float)bt + 1.0f) - 1.0f) * 0.5f));
    while ((SI + 1) * (SI + 2) / 2 <= bt) ++SI;
    while (SI * (SI + 1) / 2 > bt) --SI;
    const int SJ = bt - SI * (SI + 1) / 2;
    const int ntq = (a.nVf + MT_Q - 1) / MT_Q;
    const int I = MT_SG * SI + w;
    const int lane = threadIdx.x & 63, sr = lane >> 4, c = lane & 15;
    float4 mine = make_float4(0.f, 0.f, 0.f, 0.f);  // row 4c + sr of tile row I
    if (I < ntq) {
        const int nrow = min(MT_Q, a.nVf - I * MT_Q);
        const float4* hI = a.hvec + I * MT_Q + sr;
#pragma unroll 1
        for (int j = 0; j < MT_SG; ++j) {
            const int J = MT_SG * SJ + j;
            if (J > I) break;  // upper triangle
            const size_t tt = (size_t)I * (I + 1) / 2 + J;
            if (!((live >> (w * MT_SG + j)) & 1ull)) continue;  // below the drop threshold: not streamed
            float hx[4], hy[4], hz[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float4 h = a.hvec[J * MT_Q + 4 * c + k];
                hx[k] = h.x;
                hy[k] = h.y;
                hz[k] = h.z;
            }
            float cs[4][3];
#pragma unroll
            for (int k = 0; k < 4; ++k) cs[k][0] = cs[k][1] = cs[k][2] = 0.f;
            if constexpr (HALF) {
                const f16x4* T4 = reinterpret_cast<const f16x4*>(a.Mh + tt * MT_TILE);
                const float sc = a.tscale[tt];
#pragma unroll 1
                for (int kk = 0; 4 * kk < nrow; kk += 4) {
                    f16x4 m[4][9];
                    float4 hi[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int il = 4 * (kk + b) + sr;
#pragma unroll
                        for (int q = 0; q < 9; ++q)
                            m[b][q] = __builtin_nontemporal_load(T4 + ((size_t)il * 9 + q) * (MT_Q / 4) + c);
                        hi[b] = hI[4 * (kk + b)];
                    }
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const float m0 = (float)m[b][0][k], m1 = (float)m[b][1][k], m2 = (float)m[b][2][k];
                            const float m3 = (float)m[b][3][k], m4 = (float)m[b][4][k], m5 = (float)m[b][5][k];
                            const float m6 = (float)m[b][6][k], m7 = (float)m[b][7][k], m8 = (float)m[b][8][k];
                            r0 = fmaf(m0, hx[k], fmaf(m1, hy[k], fmaf(m2, hz[k], r0)));
                            r1 = fmaf(m3, hx[k], fmaf(m4, hy[k], fmaf(m5, hz[k], r1)));
                            r2 = fmaf(m6, hx[k], fmaf(m7, hy[k], fmaf(m8, hz[k], r2)));
                            cs[k][0] = fmaf(m0, hi[b].x, fmaf(m3, hi[b].y, fmaf(m6, hi[b].z, cs[k][0])));
                            cs[k][1] = fmaf(m1, hi[b].x, fmaf(m4, hi[b].y, fmaf(m7, hi[b].z, cs[k][1])));
                            cs[k][2] = fmaf(m2, hi[b].x, fmaf(m5, hi[b].y, fmaf(m8, hi[b].z, cs[k][2])));
                        }
                        r0 = lane_sum_w<16>(r0);
                        r1 = lane_sum_w<16>(r1);
                        r2 = lane_sum_w<16>(r2);
                        if (c == kk + b) {
                            mine.x += sc * r0;
                            mine.y += sc * r1;
                            mine.z += sc * r2;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    cs[k][0] *= sc;
                    cs[k][1] *= sc;
                    cs[k][2] *= sc;
                }
            } else {
                const f32x4* T4 = reinterpret_cast<const f32x4*>(a.Mt + tt * MT_TILE);
#pragma unroll 1
                for (int kk = 0; 4 * kk < nrow; kk += 2) {
                    f32x4 m[2][9];
                    float4 hi[2];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int il = 4 * (kk + b) + sr;
#pragma unroll
                        for (int q = 0; q < 9; ++q)
                            m[b][q] = __builtin_nontemporal_load(T4 + ((size_t)il * 9 + q) * (MT_Q / 4) + c);
                        hi[b] = hI[4 * (kk + b)];
                    }
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const float m0 = m[b][0][k], m1 = m[b][1][k], m2 = m[b][2][k];
                            const float m3 = m[b][3][k], m4 = m[b][4][k], m5 = m[b][5][k];
                            const float m6 = m[b][6][k], m7 = m[b][7][k], m8 = m[b][8][k];
                            r0 = fmaf(m0, hx[k], fmaf(m1, hy[k], fmaf(m2, hz[k], r0)));
                            r1 = fmaf(m3, hx[k], fmaf(m4, hy[k], fmaf(m5, hz[k], r1)));
                            r2 = fmaf(m6, hx[k], fmaf(m7, hy[k], fmaf(m8, hz[k], r2)));
                            cs[k][0] = fmaf(m0, hi[b].x, fmaf(m3, hi[b].y, fmaf(m6, hi[b].z, cs[k][0])));
                            cs[k][1] = fmaf(m1, hi[b].x, fmaf(m4, hi[b].y, fmaf(m7, hi[b].z, cs[k][1])));
                            cs[k][2] = fmaf(m2, hi[b].x, fmaf(m5, hi[b].y, fmaf(m8, hi[b].z, cs[k][2])));
                        }
                        r0 = lane_sum_w<16>(r0);
                        r1 = lane_sum_w<16>(r1);
                        r2 = lane_sum_w<16>(r2);
                        if (c == kk + b) {
                            mine.x += r0;
                            mine.y += r1;
                            mine.z += r2;
                        }
                    }
                }
            }
            if (I != J) {
                // column sums over the four 16-lane rows; lane (sr, c) keeps column 4c + sr
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        float v = cs[k][r];
                        v += __shfl_xor(v, 16, 64);
                        v += __shfl_xor(v, 32, 64);
                        cs[k][r] = v;
                    }
                float c0 = cs[0][0], c1 = cs[0][1], c2 = cs[0][2];
#pragma unroll
                for (int k = 1; k < 4; ++k)
                    if (sr == k) {
                        c0 = cs[k][0];
                        c1 = cs[k][1];
                        c2 = cs[k][2];
                    }
                sCol[w][j][0][4 * c + sr] = c0;
                sCol[w][j][1][4 * c + sr] = c1;
                sCol[w][j][2][4 * c + sr] = c2;
            }
        }
        const f32x4 mv = {mine.x, mine.y, mine.z, 0.0f};
        __builtin_nontemporal_store(mv, reinterpret_cast<f32x4*>(a.prow) + ((size_t)SJ * ntq + I) * MT_Q + 4 * c + sr);
    }
    __syncthreads();
    // column partials of tile column J = MT_SG SJ + w: the waves' parts in order
    const int J = MT_SG * SJ + w;
    if (J < ntq) {
        float y0 = 0.f, y1 = 0.f, y2 = 0.f;
#pragma unroll 1
        for (int ww = 0; ww < MT_SG; ++ww) {
            const int Iw = MT_SG * SI + ww;
            if (Iw > J && Iw < ntq && ((live >> (ww * MT_SG + w)) & 1ull)) {
                y0 += sCol[ww][w][0][lane];
                y1 += sCol[ww][w][1][lane];
                y2 += sCol[ww][w][2][lane];
            }
        }
        const f32x4 yv = {y0, y1, y2, 0.0f};
        __builtin_nontemporal_store(yv, reinterpret_cast<f32x4*>(a.pcol) + ((size_t)SI * ntq + J) * MT_Q + lane);
    }
}

// (H-bar^-1 h)_q for the 64 positions of tile row X (in super-tile row SX):
// the row partials prow[SJ][X], SJ <= SX, then the column partials
// pcol[SI][X], SI >= SX, of the super-tiles whose tiles are streamed (those
// of the others stay zero and are not read), wave w taking every fourth,
// FP64 sums, the four
// waves combined in a fixed order.
__global__ __launch_bounds__(256) void k_ysum(SweepArgs a) {
    __shared__ double sy[4][MT_Q][3];
    const int X = blockIdx.x;
    const int ntq = (a.nVf + MT_Q - 1) / MT_Q;
    const int ns = (ntq + MT_SG - 1) / MT_SG;
    const int SX = X / MT_SG;
    // partials k = 0 .. SX: row partials prow[k]; k = SX + 1 .. ns: column
    // partials pcol[k - 1]; outside [k0, n) they are zero (dead super-tiles)
    const int k0 = a.srange ? IX(a, a.srange[SX].x, SX + 2) : 0;
    const int n = a.srange ? IX(a, a.srange[SX].y + 1, ns + 1) + 1 : ns + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    auto at = [&](int k) -> const float4* {
        return k <= SX ? a.prow + ((size_t)k * ntq + X) * MT_Q + lane
                       : a.pcol + ((size_t)(SX + k - SX - 1) * ntq + X) * MT_Q + lane;
    };
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    int k = k0 + w;
    for (; k + 28 < n; k += 32) {  // eight loads in flight
        float4 p[8];
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) p[kb] = *at(k + 4 * kb);
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
            y0 += p[kb].x;
            y1 += p[kb].y;
            y2 += p[kb].z;
        }
    }
    for (; k < n; k += 4) {
        const float4 p = *at(k);
        y0 += p.x;
        y1 += p.y;
        y2 += p.z;
    }
    sy[w][lane][0] = y0;
    sy[w][lane][1] = y1;
    sy[w][lane][2] = y2;
    __syncthreads();
    const int q = X * MT_Q + threadIdx.x;
    if (threadIdx.x < MT_Q && q < a.nVf) {
        float y[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            y[r] = (float)(((sy[0][threadIdx.x][r] + sy[1][threadIdx.x][r]) + sy[2][threadIdx.x][r]) + sy[3][threadIdx.x][r]);
        a.yq[q] = make_float4(y[0], y[1], y[2], 0.0f);
    }
}

// Sixteen lanes per row (16 rows per 256-thread block), rows in position
// order when every row is swept (neighbouring rows then share tet and
// position lines) or from a.list (free indices).  The reduced gradient comes
// from a.yq; the row's lanes take its incident tets for the Hessian term,
// with Phi_{f,b} = R_b U-bar_{f,b} R_f^T from the row's one-ring U-bar rows
// (contiguous per row, addressed by the incidence's slot word), summed over
// the 16 lanes by DPP; the row's first lane solves.
// LIN (adjoint): the same local system of H(x*) y = rhs, with the linear
// residual r = H y - rhs in place of g (its rest-frame form behind a.yq), the
// Hessian at a.u = x*, and the update applied to y.
constexpr int EX_LANES = 16;
template <bool LIN>
__global__ __launch_bounds__(256) void k_exact(SweepArgs a) {
    const int lane = threadIdx.x & (EX_LANES - 1);
    const int row = xcd_remap(blockIdx.x, gridDim.x) * (256 / EX_LANES) + (threadIdx.x / EX_LANES);
    const int nidx = a.list ? a.n_list : a.nVf;
    if (row >= nidx) return;  // the row's 16 lanes
    int f, v, qf;
    if (a.list) {
        f = IX(a, a.list[row], a.nVf);
        v = IX(a, a.free_ids[f], a.nV);
        qf = IX(a, a.qpos[v], a.nVf);
    } else {
        qf = row;
        f = IX(a, a.qfree[qf], a.nVf);
        v = IX(a, a.qvert[qf], a.nV);
    }
    const d4 uv = a.u[v];
    if (!LIN && !body_on(a, f)) {
        if (lane == 0 && !a.in_place) a.unext[v] = uv;  // a stopped body's Jacobi buffer carried over
        return;
    }
    float Ri[9];
    load_rot(a.R, v, Ri);
    // Hessian term over the incident tets, one per lane
    float A9[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int n = a.inc_n[f];
    for (int j = lane; j < n; j += EX_LANES) {
        const int4 e = IX_INC(a, a.inc4[(size_t)f * a.maxi + j]);
        const uint32_t sl = a.incslot[(size_t)f * a.maxi + j];
        const int c = e.x & 3;
        Tet T;
        load_tet_inc(a.tet, e, v, T);
        float H[9], cH[9];
        Kin<float> K;
        dispgrad(a.u, T, H);
        kinematics(H, K, cH);
        float dF[3][9];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 9; ++q) dF[d][q] = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t sb = (sl >> (8 * b)) & 0xFFu;
            float Phi[9];
            if (sb == SLOT_SELF) {
#pragma unroll
                for (int q = 0; q < 9; ++q) Phi[q] = (q % 4 == 0) ? 1.0f : 0.0f;
            } else if (sb == SLOT_NONE) {
#pragma unroll
                for (int q = 0; q < 9; ++q) Phi[q] = 0.0f;
            } else {
                float Ub[9], Rb[9];
                const int sk = IX(a, sb, a.K);
#pragma unroll
                for (int q = 0; q < 9; ++q) Ub[q] = a.Uring[((size_t)f * 9 + q) * a.K + sk];
                load_rot(a.R, T.id[b], Rb);
                corotate(Ub, Ri, Rb, Phi);
            }
            float gnb[3];
            gradN(T.D, b, gnb);
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj) dF[d][3 * i + jj] = fmaf(Phi[3 * i + d], gnb[jj], dF[d][3 * i + jj]);
        }
        float gnc[3];
        gradN(T.D, c, gnc);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float dP[9];
            snh_dstress(K.F, K.C, 1.0f + K.Jm1, T.vmu, T.vlam, dF[d], dP);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                A9[3 * i + d] += dP[3 * i] * gnc[0] + dP[3 * i + 1] * gnc[1] + dP[3 * i + 2] * gnc[2];
        }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) A9[q] = lane_sum_w<EX_LANES>(A9[q]);
    if (lane == 0) {
        // b = R_f B_f^-1 y
        float Bi[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) Bi[q] = a.Binv[(size_t)qf * 9 + q];
        const float4 y4 = a.yq[qf];
        const float yy[3] = {y4.x, y4.y, y4.z};
        float by[3], b[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) by[i] = Bi[3 * i] * yy[0] + Bi[3 * i + 1] * yy[1] + Bi[3 * i + 2] * yy[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) b[i] = Ri[3 * i] * by[0] + Ri[3 * i + 1] * by[1] + Ri[3 * i + 2] * by[2];
        const float m = LIN ? a.mh2[v] : (float)a.zu[v].w;
        float A[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) A[3 * i + jj] = 0.5f * (A9[3 * i + jj] + A9[3 * jj + i]);
        A[0] += m; A[4] += m; A[8] += m;
        float gd[3] = {0.f, 0.f, 0.f}, Hb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        barrier_terms(a, v, uv, gd, Hb);
        A[0] += Hb[0]; A[1] += Hb[1]; A[2] += Hb[2];
        A[3] += Hb[1]; A[4] += Hb[3]; A[5] += Hb[4];
        A[6] += Hb[2]; A[7] += Hb[4]; A[8] += Hb[5];
        float dx[3];
        local_solve(A, b, dx);
        float st[3] = {a.omega * dx[0], a.omega * dx[1], a.omega * dx[2]};
        if (LIN) {
            const float4 yv = a.ly[v];
            float4* out = a.in_place ? const_cast<float4*>(a.ly) : a.lynext;
            out[v] = make_float4(yv.x + st[0], yv.y + st[1], yv.z + st[2], 0.0f);
        } else {
            clamp_step(a, v, uv, st);
            d4* out = a.in_place ? const_cast<d4*>(a.u) : a.unext;
            out[v] = make_d4(uv.x + st[0], uv.y + st[1], uv.z + st[2], 0.0);
        }
    }
}

// thetabar_t -= sum_c y_c . (V_t P(F_t) grad N_c) at the displacement u:
// the derivative of the step's optimality condition with respect to
// log E_t is the element's elastic force, since mu and lambda scale with E.
__global__ void k_param_grad(const float4* __restrict__ tet, int nT, const d4* __restrict__ u,
                             const float4* __restrict__ y, double* __restrict__ thbar) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nT) return;
    Tet T;
    load_tet(tet, t, T);
    float H[9], cH[9], P[9];
    Kin<float> K;
    dispgrad(u, T, H);
    kinematics(H, K, cH);
    snh_stress_H(H, K, cH, T.vmu, T.vlam, P);
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float gn[3];
        gradN(T.D, c, gn);
        const float4 yc = y[T.id[c]];
        acc += yc.x * (P[0] * gn[0] + P[1] * gn[1] + P[2] * gn[2]) +
               yc.y * (P[3] * gn[0] + P[4] * gn[1] + P[5] * gn[2]) +
               yc.z * (P[6] * gn[0] + P[7] * gn[1] + P[8] * gn[2]);
    }
    thbar[t] -= (double)acc;
}

// Cotangents of the previous step's inputs and the next right-hand side:
// xbar <- m/h^2 y - vbar/h, vbar <- h m/h^2 y, rhs <- xbar + vbar/h
// (zero at pinned vertices, where m/h^2 is stored as 0).
__global__ void k_adj_vec(int nV, const float* __restrict__ mh2, const float4* __restrict__ y,
                          float4* __restrict__ xbar, float4* __restrict__ vbar, float4* __restrict__ rhs,
                          float h) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const float m = mh2[v];
    const float4 yv = y[v], vb = vbar[v];
    const float ih = 1.0f / h;
    float4 xn, vn;
    if (m > 0.0f) {
        xn = make_float4(m * yv.x - vb.x * ih, m * yv.y - vb.y * ih, m * yv.z - vb.z * ih, 0.0f);
        vn = make_float4(h * m * yv.x, h * m * yv.y, h * m * yv.z, 0.0f);
    } else {
        xn = make_float4(0.f, 0.f, 0.f, 0.f);
        vn = xn;
    }
    xbar[v] = xn;
    vbar[v] = vn;
    rhs[v] = make_float4(xn.x + vn.x * ih, xn.y + vn.y * ih, xn.z + vn.z * ih, 0.0f);
}

// Per-body |g|^2 in FP64, in two fixed-order passes so the value does not
// depend on the other bodies: block c sums chunk c (at most CHUNK free
// vertices of one body, grouped by seg_idx), then one thread per body adds
// its chunks in order.
constexpr int CHUNK = 1024;
__global__ __launch_bounds__(256) void k_chunk_norm2(const int* __restrict__ chunk_lo, const int* __restrict__ chunk_hi,
                                                     const int* __restrict__ seg_idx, const int* __restrict__ free_ids,
                                                     const float4* __restrict__ g, double* __restrict__ r2c) {
    __shared__ double s[256];
    const int c = blockIdx.x;
    const int lo = chunk_lo[c], hi = chunk_hi[c];
    double e = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += 256) {
        const float4 q = g[free_ids[seg_idx[i]]];
        e += (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) r2c[c] = s[0];
}

__global__ void k_seg_finish(int nb, const int* __restrict__ body_chunk_off, const double* __restrict__ r2c,
                             double* __restrict__ r2) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    double t = 0.0;
    for (int c = body_chunk_off[b]; c < body_chunk_off[b + 1]; ++c) t += r2c[c];
    r2[b] = t;
}

// A residual check inside a step, in two launches: per chunk the |g|^2 and
// |u - u_prev|^2 partials (the |g|^2 sums as in k_chunk_norm2), then one
// block for the per-body sums (each body's chunks in order, as in
// k_seg_finish), the sweep counts of the bodies that ran, the stop flags
// (|g_b| <= tol |g_b(x0)|), the count of bodies still on, and the update norm
// (partials in a fixed order).
__global__ __launch_bounds__(256) void k_check_chunks(const int* __restrict__ chunk_lo, const int* __restrict__ chunk_hi,
                                                      const int* __restrict__ seg_idx, const int* __restrict__ free_ids,
                                                      const float4* __restrict__ g, const d4* __restrict__ u,
                                                      const d4* __restrict__ uprev, double* __restrict__ r2c,
                                                      double* __restrict__ dx2c) {
    __shared__ double s[256], t[256];
    const int c = blockIdx.x;
    const int lo = chunk_lo[c], hi = chunk_hi[c];
    double e = 0.0, f = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += 256) {
        const int v = free_ids[seg_idx[i]];
        const float4 q = g[v];
        e += (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z;
        const double dx = u[v].x - uprev[v].x, dy = u[v].y - uprev[v].y, dz = u[v].z - uprev[v].z;
        f += dx * dx + dy * dy + dz * dz;
    }
    s[threadIdx.x] = e;
    t[threadIdx.x] = f;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s[threadIdx.x] += s[threadIdx.x + o];
            t[threadIdx.x] += t[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        r2c[c] = s[0];
        dx2c[c] = t[0];
    }
}

__global__ __launch_bounds__(256) void k_check_finish(int nb, const int* __restrict__ body_chunk_off,
                                                      const double* __restrict__ r2c, double* __restrict__ r2,
                                                      const double* __restrict__ r0sq, double tol2, int* __restrict__ on,
                                                      int* __restrict__ sweeps, int k, int* __restrict__ n_active,
                                                      int n_chunks, const double* __restrict__ dx2c,
                                                      double* __restrict__ dx2) {
    __shared__ int cnt[256];
    __shared__ double sh[256];
    int c = 0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        double t = 0.0;
        for (int q = body_chunk_off[b]; q < body_chunk_off[b + 1]; ++q) t += r2c[q];
        r2[b] = t;
        if (on[b]) {
            sweeps[b] += k;
            if (t <= tol2 * r0sq[b]) on[b] = 0;
        }
        c += on[b];
    }
    double d = 0.0;
    for (int i = threadIdx.x; i < n_chunks; i += 256) d += dx2c[i];
    cnt[threadIdx.x] = c;
    sh[threadIdx.x] = d;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            cnt[threadIdx.x] += cnt[threadIdx.x + o];
            sh[threadIdx.x] += sh[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        n_active[0] = cnt[0];
        dx2[0] = sh[0];
    }
}

// Start of a step: r0^2 per body, every body with a non-zero residual on.
__global__ __launch_bounds__(256) void k_mask_init(int nb, const double* __restrict__ r2, double* __restrict__ r0sq,
                                                   int* __restrict__ on, int* __restrict__ sweeps,
                                                   int* __restrict__ n_active) {
    __shared__ int cnt[256];
    int c = 0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        r0sq[b] = r2[b];
        on[b] = r2[b] > 0.0 ? 1 : 0;
        sweeps[b] = 0;
        c += on[b];
    }
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) n_active[0] = cnt[0];
}

// Per-block FP64 partial sums of |w_v|^2 over free vertices.
__global__ __launch_bounds__(256) void k_norm2(int nVf, const int* __restrict__ free_ids,
                                               const float4* __restrict__ w, double* __restrict__ partial) {
    __shared__ double s[256];
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (f < nVf) {
        const float4 q = w[free_ids[f]];
        e = (double)q.x * q.x + (double)q.y * q.y + (double)q.z * q.z;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// Copies updated positions of the listed vertices from unext into u.
__global__ void k_commit(SweepArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n_list) return;
    const int v = a.free_ids[a.list[idx]];
    const_cast<d4*>(a.u)[v] = a.unext[v];
}

// Backtracking: unext <- u + t (unext - u) on free vertices.
__global__ void k_blend(SweepArgs a, float t) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= a.nVf) return;
    const int v = a.free_ids[f];
    const d4 x = a.u[v], y = a.unext[v];
    const double tt = t;
    a.unext[v] = make_d4(x.x + tt * (y.x - x.x), x.y + tt * (y.y - x.y), x.z + tt * (y.z - x.z), 0.0);
}

// Fixed-order sum of n per-block partials into out[0] (one block).
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ in, int n, double* out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += in[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// z = xhat + h vhat + h^2 g on free vertices (displacement form; w = m/h^2),
// x0 = xhat.
__global__ void k_predict(int nV, const d4* __restrict__ uhat, const float4* __restrict__ vhat,
                          const float* __restrict__ mh2, float h, float g0, float g1, float g2,
                          d4* __restrict__ u, d4* __restrict__ unext, d4* __restrict__ zu) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const d4 x = uhat[v];
    u[v] = x;
    unext[v] = x;
    const float m = mh2[v];
    if (m > 0.0f) {
        const float4 vv = vhat[v];
        const double hd = h, h2 = hd * hd;
        zu[v] = make_d4(x.x + hd * vv.x + h2 * g0, x.y + hd * vv.y + h2 * g1, x.z + hd * vv.z + h2 * g2, m);
    } else {
        zu[v] = make_d4(x.x, x.y, x.z, 0.0);
    }
}

// v = (x - xhat) / h ; xhat <- x
__global__ void k_velocity(int nV, const d4* __restrict__ u, d4* __restrict__ uhat, float4* __restrict__ vhat,
                           double inv_h) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const d4 x = u[v], x0 = uhat[v];
    vhat[v] = make_float4((float)((x.x - x0.x) * inv_h), (float)((x.y - x0.y) * inv_h), (float)((x.z - x0.z) * inv_h),
                          0.0f);
    uhat[v] = x;
}

// Incremental potential: per-tet V Psi(F) + per-free-vertex inertia and
// barrier terms, FP64 per-block partials.
__global__ __launch_bounds__(256) void k_energy(SweepArgs a, int nT) {
    __shared__ double s[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < nT) {
        Tet T;
        load_tet(a.tet, i, T);
        float H[9], cH[9];
        Kin<float> K;
        dispgrad(a.u, T, H);
        kinematics(H, K, cH);
        e += (double)snh_psi_H(H, K, cH, T.vmu, T.vlam);
    }
    if (i < a.nVf) {
        const int v = a.free_ids[i];
        const d4 uv = a.u[v], zv = a.zu[v];
        const double d0 = uv.x - zv.x, d1 = uv.y - zv.y, d2 = uv.z - zv.z;
        e += 0.5 * zv.w * (d0 * d0 + d1 * d1 + d2 * d2);
        const float4 X = a.X[v];
        const double x[3] = {(double)X.x + uv.x, (double)X.y + uv.y, (double)X.z + uv.z};
        for (int p = 0; p < JGS2_MAX_PLANES; ++p) {
            if (p >= a.n_planes) break;
            const double d = a.planes[p][0] * x[0] + a.planes[p][1] * x[1] + a.planes[p][2] * x[2] - a.planes[p][3];
            e += (d <= 0.0) ? INFINITY : (double)a.kappa * barrier<double>(d, (double)a.d_hat);
        }
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[blockIdx.x] = s[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int n_blocks_for(const SweepArgs& a) {
    const int n = a.list ? a.n_list : a.nVf;
    return (n + VPB - 1) / VPB;
}

void launch_phase1(jgs2_solver* s, const SweepArgs& a, bool want_R, bool gate) {
    const int nb = n_blocks_for(a);
    if (nb == 0) return;
    if (gate && !a.one_body && a.body_on != nullptr)
        launch(s, JGS2_K_PHASE1, k_phase1<true>, dim3(nb), dim3(BLOCK), a, want_R ? 1 : 0);
    else
        launch(s, JGS2_K_PHASE1, k_phase1<false>, dim3(nb), dim3(BLOCK), a, want_R ? 1 : 0);
}

void launch_phase2_cubature(jgs2_solver* s, const SweepArgs& a) {
    const int nb = n_blocks_for(a);
    if (nb == 0) return;
    launch(s, JGS2_K_PHASE2, k_phase2_cubature, dim3(nb), dim3(BLOCK), a);
}

// Launch of a plain or linear sweep kernel in the tuned shape (W lanes per
// vertex, BLK threads per block).
// KIND 0: plain, 1: linear (adjoint), 2: damper.
template <int KIND, int W, int BLK>
static void launch_plain_t(jgs2_solver* s, const SweepArgs& a) {
    constexpr bool LIN = KIND == 1;
    constexpr int NV = BLK / W;
    const int n = a.list ? a.n_list : a.nVf;
    const int nb = (n + NV - 1) / NV;
    if (nb == 0) return;
    const dim3 g(nb), b(BLK);
    if (KIND == 2) {
        if (a.one_body) {
            if (a.nt_records) launch(s, JGS2_K_DAMPER, k_damper<W, BLK, true, true>, g, b, a);
            else launch(s, JGS2_K_DAMPER, k_damper<W, BLK, true, false>, g, b, a);
        } else {
            if (a.nt_records) launch(s, JGS2_K_DAMPER, k_damper<W, BLK, false, true>, g, b, a);
            else launch(s, JGS2_K_DAMPER, k_damper<W, BLK, false, false>, g, b, a);
        }
    } else if (LIN) {
        if (a.nt_records) launch(s, JGS2_K_LINEAR, k_linear<W, BLK, true>, g, b, a);
        else launch(s, JGS2_K_LINEAR, k_linear<W, BLK, false>, g, b, a);
    } else if (a.one_body) {
        if (a.nt_records) launch(s, JGS2_K_PLAIN, k_plain<W, BLK, true, true>, g, b, a);
        else launch(s, JGS2_K_PLAIN, k_plain<W, BLK, true, false>, g, b, a);
    } else {
        if (a.nt_records) launch(s, JGS2_K_PLAIN, k_plain<W, BLK, false, true>, g, b, a);
        else launch(s, JGS2_K_PLAIN, k_plain<W, BLK, false, false>, g, b, a);
    }
}

template <int KIND, int W>
static void launch_plain_w(jgs2_solver* s, const SweepArgs& a) {
    switch (s->tune_block) {
        case 64: launch_plain_t<KIND, W, 64>(s, a); break;
        case 128: launch_plain_t<KIND, W, 128>(s, a); break;
        case 512: launch_plain_t<KIND, W, 512>(s, a); break;
        default: launch_plain_t<KIND, W, 256>(s, a); break;
    }
}

template <int KIND>
static void launch_plain_any(jgs2_solver* s, const SweepArgs& a) {
    switch (s->tune_lpv) {
        case 4: launch_plain_w<KIND, 4>(s, a); break;
        case 8: launch_plain_w<KIND, 8>(s, a); break;
        case 16: launch_plain_w<KIND, 16>(s, a); break;
        default: launch_plain_w<KIND, 32>(s, a); break;
    }
}

void launch_plain(jgs2_solver* s, const SweepArgs& a) { launch_plain_any<0>(s, a); }

// Grid: the resident block count (occupancy x compute units), or fewer when
// the largest colour has fewer row blocks.  The block is 256 threads whatever
// the tuned block size (rows are independent: the result does not depend on
// it), the lanes per vertex are the tuned ones (they fix the summation order).
template <int W>
static int launch_persistent_w(jgs2_solver* s, const SweepArgs& a, int k) {
    constexpr int BLK = 256, NV = BLK / W;
    void (*kern)(SweepArgs, int, const int*, int, d4*) =
        a.one_body ? (a.nt_records ? k_plain_persistent<W, BLK, true, true> : k_plain_persistent<W, BLK, true, false>)
                   : (a.nt_records ? k_plain_persistent<W, BLK, false, true> : k_plain_persistent<W, BLK, false, false>);
    int per_cu = 0;
    int r = hip_check(s, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, BLK, 0),
                      "persistent occupancy");
    if (r != JGS2_OK) return r;
    int most = 0;
    for (int c = 0; c < s->n_colors; ++c) most = std::max(most, s->col_off[c + 1] - s->col_off[c]);
    // a multiple of 8 (one share per XCD), at least 8
    const int grid = std::max(8, std::min(per_cu * s->n_cus, (most + NV - 1) / NV) / 8 * 8);
    SweepArgs aa = a;
    int kk = k, nc = s->n_colors;
    const int* co = s->d_coloff;
    d4* up = s->d_uprev;
    void* args[] = {(void*)&aa, (void*)&kk, (void*)&co, (void*)&nc, (void*)&up};
    return hip_check(s, hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(BLK), args, 0, s->stream),
                     "persistent cooperative launch");
}

int launch_plain_persistent(jgs2_solver* s, const SweepArgs& a, int k) {
    switch (s->tune_lpv) {
        case 4: return launch_persistent_w<4>(s, a, k);
        case 8: return launch_persistent_w<8>(s, a, k);
        case 16: return launch_persistent_w<16>(s, a, k);
        default: return launch_persistent_w<32>(s, a, k);
    }
}

void launch_linear(jgs2_solver* s, const SweepArgs& a) { launch_plain_any<1>(s, a); }

void launch_damper(jgs2_solver* s, const SweepArgs& a) { launch_plain_any<2>(s, a); }

// h, the tile products and their per-position sums.
void launch_reduced_gradient(jgs2_solver* s, const SweepArgs& a) {
    if (a.nVf == 0) return;
    launch(s, JGS2_K_HVEC, k_hvec, dim3((a.nVf + 255) / 256), dim3(256), a);
    const int ns = (a.nVf + MT_Q * MT_SG - 1) / (MT_Q * MT_SG);
    const int nb = a.slist ? a.n_slive : ns * (ns + 1) / 2;
    if (nb > 0) {
        if (s->tiles_fp16)
            launch(s, JGS2_K_SYMV, k_symv<true>, dim3((unsigned)nb), dim3(64 * MT_SG), a);
        else
            launch(s, JGS2_K_SYMV, k_symv<false>, dim3((unsigned)nb), dim3(64 * MT_SG), a);
    }
    launch(s, JGS2_K_YSUM, k_ysum, dim3((a.nVf + MT_Q - 1) / MT_Q), dim3(256), a);
}

#ifdef JGS2_BOUNDS_CHECK
// Records a failed check (index 1 of extent 0) from one lane, touching no buffer.
__global__ void k_bounds_selftest(unsigned long long* rec) {
    if (threadIdx.x == 0) bounds_fail(rec, 1, 0, __LINE__);
}
#endif

void launch_bounds_selftest(jgs2_solver* s) {
#ifdef JGS2_BOUNDS_CHECK
    hipLaunchKernelGGL(k_bounds_selftest, dim3(1), dim3(64), 0, s->stream, s->d_bounds);
#else
    (void)s;
#endif
}

// FP32 tiles to FP16, one block per tile: entry x inv[tile], rounded to nearest.
__global__ __launch_bounds__(256) void k_tiles_to_fp16(const float* __restrict__ Mt, _Float16* __restrict__ Mh,
                                                       const float* __restrict__ inv) {
    const size_t t = blockIdx.x;
    const float sc = inv[t];
    const float4* src = reinterpret_cast<const float4*>(Mt + t * MT_TILE);
    f16x4* dst = reinterpret_cast<f16x4*>(Mh + t * MT_TILE);
    for (int i = threadIdx.x; i < (int)(MT_TILE / 4); i += 256) {
        const float4 v = src[i];
        const f16x4 h = {(_Float16)(v.x * sc), (_Float16)(v.y * sc), (_Float16)(v.z * sc), (_Float16)(v.w * sc)};
        dst[i] = h;
    }
}

void launch_tiles_to_fp16(jgs2_solver* s, const float* Mt, _Float16* Mh, const float* inv, size_t n_tiles) {
    if (n_tiles == 0) return;
    hipLaunchKernelGGL(k_tiles_to_fp16, dim3((unsigned)n_tiles), dim3(256), 0, s->stream, Mt, Mh, inv);
}

// Sixteen lanes per row, 16 rows per block.
void launch_exact(jgs2_solver* s, const SweepArgs& a) {
    const int n = a.list ? a.n_list : a.nVf;
    if (n == 0) return;
    constexpr int R = 256 / EX_LANES;
    launch(s, JGS2_K_EXACT, k_exact<false>, dim3((n + R - 1) / R), dim3(256), a);
}

void launch_exact_linear(jgs2_solver* s, const SweepArgs& a) {
    const int n = a.list ? a.n_list : a.nVf;
    if (n == 0) return;
    constexpr int R = 256 / EX_LANES;
    launch(s, JGS2_K_EXACT, k_exact<true>, dim3((n + R - 1) / R), dim3(256), a);
}

// Rotation pass in a fixed shape (8 lanes per row, 64 rows per block): its
// cost is the gather plus one polar decomposition per row, which this shape
// runs 64 to a wave.
void launch_rotations(jgs2_solver* s, const SweepArgs& a) {
    constexpr int W = 8, BLK = 512, NV = BLK / W;
    const int nb = (a.nVf + NV - 1) / NV;
    if (nb == 0) return;
    const dim3 g(nb), b(BLK);
    if (a.one_body) {
        if (a.nt_records) launch(s, JGS2_K_ROT, k_rot<W, BLK, true, true>, g, b, a);
        else launch(s, JGS2_K_ROT, k_rot<W, BLK, true, false>, g, b, a);
    } else {
        if (a.nt_records) launch(s, JGS2_K_ROT, k_rot<W, BLK, false, true>, g, b, a);
        else launch(s, JGS2_K_ROT, k_rot<W, BLK, false, false>, g, b, a);
    }
}

void launch_param_grad(jgs2_solver* s, const d4* u, const float4* y, double* thbar) {
    launch(s, JGS2_K_PARAMGRAD, k_param_grad, dim3((s->nT + 255) / 256), dim3(256), (const float4*)s->d_tet, s->nT,
           u, y, thbar);
}

void launch_adj_vec(jgs2_solver* s, const float4* y, float4* xbar, float4* vbar, float4* rhs) {
    launch(s, JGS2_K_ADJVEC, k_adj_vec, dim3((s->nV + 255) / 256), dim3(256), s->nV, (const float*)s->d_mh2, y,
           xbar, vbar, rhs, (float)s->p.dt);
}

void launch_norm2(jgs2_solver* s, const float4* w) {
    launch(s, JGS2_K_REDUCE, k_norm2, dim3((s->nVf + 255) / 256), dim3(256), s->nVf, (const int*)s->d_free, w,
           s->d_partial);
}

void launch_seg_norm2(jgs2_solver* s) {
    if (s->n_chunks > 0)
        launch(s, JGS2_K_REDUCE, k_chunk_norm2, dim3(s->n_chunks), dim3(256), (const int*)s->d_chunk_lo,
               (const int*)s->d_chunk_hi, (const int*)s->d_seg_idx, (const int*)s->d_free, (const float4*)s->d_g,
               s->d_r2c);
    launch(s, JGS2_K_REDUCE, k_seg_finish, dim3((s->n_bodies + 255) / 256), dim3(256), s->n_bodies,
           (const int*)s->d_body_chunk_off, (const double*)s->d_r2c, s->d_r2);
}

int seg_chunk_size() { return CHUNK; }

void launch_check(jgs2_solver* s, int k) {
    if (s->n_chunks > 0)
        launch(s, JGS2_K_REDUCE, k_check_chunks, dim3(s->n_chunks), dim3(256), (const int*)s->d_chunk_lo,
               (const int*)s->d_chunk_hi, (const int*)s->d_seg_idx, (const int*)s->d_free, (const float4*)s->d_g,
               (const d4*)s->d_u, (const d4*)s->d_uprev, s->d_r2c, s->d_dx2c);
    const double tol2 = s->p.rel_tol * s->p.rel_tol;
    launch(s, JGS2_K_REDUCE, k_check_finish, dim3(1), dim3(256), s->n_bodies, (const int*)s->d_body_chunk_off,
           (const double*)s->d_r2c, s->d_r2, (const double*)s->d_r0sq, tol2, s->d_body_on, s->d_body_sweeps, k,
           s->d_nactive, s->n_chunks, (const double*)s->d_dx2c, s->d_dx2);
}

void launch_mask_init(jgs2_solver* s) {
    launch(s, JGS2_K_REDUCE, k_mask_init, dim3(1), dim3(256), s->n_bodies, (const double*)s->d_r2, s->d_r0sq,
           s->d_body_on, s->d_body_sweeps, s->d_nactive);
}

void launch_commit(jgs2_solver* s, const SweepArgs& a) {
    if (a.n_list == 0) return;
    launch(s, JGS2_K_COMMIT, k_commit, dim3((a.n_list + 255) / 256), dim3(256), a);
}

void launch_blend(jgs2_solver* s, const SweepArgs& a, float t) {
    launch(s, JGS2_K_COMMIT, k_blend, dim3((a.nVf + 255) / 256), dim3(256), a, t);
}

void launch_reduce(jgs2_solver* s, int n) {
    launch(s, JGS2_K_REDUCE, k_reduce, dim3(1), dim3(256), (const double*)s->d_partial, n, s->d_red);
}

void launch_reduce_into(jgs2_solver* s, const double* in, int n, double* out) {
    launch(s, JGS2_K_REDUCE, k_reduce, dim3(1), dim3(256), in, n, out);
}

void launch_predict(jgs2_solver* s, float h, const float* grav) {
    launch(s, JGS2_K_PREDICT, k_predict, dim3((s->nV + 255) / 256), dim3(256), s->nV, (const d4*)s->d_uhat,
           (const float4*)s->d_vhat, (const float*)s->d_mh2, h, grav[0], grav[1], grav[2], s->d_u, s->d_unext,
           s->d_zu);
}

void launch_velocity(jgs2_solver* s, float h) {
    launch(s, JGS2_K_VELOCITY, k_velocity, dim3((s->nV + 255) / 256), dim3(256), s->nV, (const d4*)s->d_u,
           s->d_uhat, s->d_vhat, 1.0 / (double)h);
}

void launch_energy(jgs2_solver* s, const SweepArgs& a, int nT) {
    const int n = nT > a.nVf ? nT : a.nVf;
    launch(s, JGS2_K_ENERGY, k_energy, dim3((n + 255) / 256), dim3(256), a, nT);
}

}  // namespace jgs2
