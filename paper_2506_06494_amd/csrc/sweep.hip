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
// All arrays of vertices are SoA [component][vertex] in FP32; positions are
// stored as displacements u = x - X from the rest shape, so that
// H = F - I = sum_a u_a (grad N_a)^T keeps full FP32 precision, and the
// stress is evaluated from H without cancelling O(mu) terms.
#include "jgs2_internal.h"
#include "jgs2_math.h"

namespace jgs2 {

__device__ __forceinline__ int xcd_remap(int i, int nb) {
    const int x = i & 7, j = i >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ float lane_sum(float v) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, LPV);
    return v;
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

// grad N of corner c: rows of Dm^-1 for corners 1..3, minus their sum for 0.
__device__ __forceinline__ void gradN(const float* D, int c, float* gn) {
    if (c == 0) {
        gn[0] = -(D[0] + D[3] + D[6]);
        gn[1] = -(D[1] + D[4] + D[7]);
        gn[2] = -(D[2] + D[5] + D[8]);
    } else {
        gn[0] = D[3 * (c - 1)]; gn[1] = D[3 * (c - 1) + 1]; gn[2] = D[3 * (c - 1) + 2];
    }
}

// H = F - I = [u1-u0, u2-u0, u3-u0] Dm^-1 (displacement gradient)
__device__ __forceinline__ void dispgrad(const float* __restrict__ u, int nV, const Tet& T, float* F) {
    float du[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float u0 = u[i * nV + T.id[0]];
#pragma unroll
        for (int k = 0; k < 3; ++k) du[k][i] = u[i * nV + T.id[k + 1]] - u0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            F[3 * i + j] = du[0][i] * T.D[j] + du[1][i] * T.D[3 + j] + du[2][i] * T.D[6 + j];
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

__device__ __forceinline__ void barrier_terms(const SweepArgs& a, int v, float* g, float* H6) {
    const float x0 = a.X[v] + a.u[v], x1 = a.X[a.nV + v] + a.u[a.nV + v], x2 = a.X[2 * a.nV + v] + a.u[2 * a.nV + v];
    for (int p = 0; p < a.n_planes; ++p) {
        const float* pl = a.planes[p];
        const float d = pl[0] * x0 + pl[1] * x1 + pl[2] * x2 - pl[3];
        if (d < a.d_hat && d > 0.0f) {
            const float b1 = a.kappa * barrier_d1(d, a.d_hat);
            g[0] += b1 * pl[0]; g[1] += b1 * pl[1]; g[2] += b1 * pl[2];
            if (H6) {
                const float b2 = a.kappa * barrier_d2(d, a.d_hat);
                H6[0] += b2 * pl[0] * pl[0]; H6[1] += b2 * pl[0] * pl[1]; H6[2] += b2 * pl[0] * pl[2];
                H6[3] += b2 * pl[1] * pl[1]; H6[4] += b2 * pl[1] * pl[2]; H6[5] += b2 * pl[2] * pl[2];
            }
        }
    }
}

__device__ __forceinline__ void block_partial(double val, bool lane0, double* partial) {
    __shared__ double sp[VPB];
    const int vloc = threadIdx.x / LPV;
    if (lane0) sp[vloc] = val;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < VPB; ++i) s += sp[i];
        partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Phase 1: assembled gradient g_a (elastic + inertia + barrier), the
// volume-weighted mean deformation gradient of the incident tets and its
// closest rotation R_a; per-block partial sums of |g|^2 (FP64).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_phase1(SweepArgs a, int want_R) {
    const int lane = threadIdx.x % LPV;
    const int vloc = threadIdx.x / LPV;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int idx = blk * VPB + vloc;
    const int nidx = a.list ? a.n_list : a.nVf;
    const bool active = idx < nidx;
    const int f = active ? (a.list ? a.list[idx] : idx) : 0;
    float g[3] = {0.f, 0.f, 0.f}, Fs[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (active) {
        const int n = a.inc_n[f];
        for (int j = lane; j < n; j += LPV) {
            const int pk = a.inc[(size_t)f * a.maxi + j];
            const int t = pk >> 2, c = pk & 3;
            Tet T;
            load_tet(a.tet, t, T);
            float H[9], cH[9], P[9], gn[3];
            Kin<float> K;
            dispgrad(a.u, a.nV, T, H);
            kinematics(H, K, cH);
            snh_stress_H(H, K, cH, T.vmu, T.vlam, P);
            gradN(T.D, c, gn);
#pragma unroll
            for (int i = 0; i < 3; ++i) g[i] += P[3 * i] * gn[0] + P[3 * i + 1] * gn[1] + P[3 * i + 2] * gn[2];
#pragma unroll
            for (int i = 0; i < 9; ++i) Fs[i] += T.vol * K.F[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = lane_sum(g[i]);
    if (want_R) {
#pragma unroll
        for (int i = 0; i < 9; ++i) Fs[i] = lane_sum(Fs[i]);
    }
    double gsq = 0.0;
    if (active && lane == 0) {
        const int v = a.free_ids[f];
        const float m = a.mh2[v];
#pragma unroll
        for (int i = 0; i < 3; ++i) g[i] += m * (a.u[i * a.nV + v] - a.zu[i * a.nV + v]);
        barrier_terms(a, v, g, nullptr);
#pragma unroll
        for (int i = 0; i < 3; ++i) a.g[i * a.nV + v] = g[i];
        gsq = (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
        if (want_R) {
            float R[9];
            closest_rotation(Fs, R);
#pragma unroll
            for (int i = 0; i < 9; ++i) a.R[i * a.nV + v] = R[i];
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
__global__ __launch_bounds__(BLOCK) void k_phase2_cubature(SweepArgs a) {
    __shared__ float sPhi[VPB][KMAX][9];
    const int lane = threadIdx.x % LPV;
    const int vloc = threadIdx.x / LPV;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int idx = blk * VPB + vloc;
    const int nidx = a.list ? a.n_list : a.nVf;
    const bool active = idx < nidx;
    const int f = active ? (a.list ? a.list[idx] : idx) : 0;
    const int v = a.free_ids[f];
    float Ri[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Ri[i] = active ? a.R[i * a.nV + v] : 0.0f;
    float A6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, b[3] = {0.f, 0.f, 0.f};

    // one-ring rows: Phi_{i,a} into LDS, gradient projection
    const int nr = active ? a.ring_n[f] : 0;
    for (int k = lane; k < nr; k += LPV) {
        const int av = a.ring[(size_t)f * a.K + k];
        float U[9], Ra[9], T9[9], Phi[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) U[q] = a.Uring[((size_t)f * 9 + q) * a.K + k];
#pragma unroll
        for (int q = 0; q < 9; ++q) Ra[q] = a.R[q * a.nV + av];
        // T9 = U R_i^T ; Phi = R_a T9
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
#pragma unroll
        for (int q = 0; q < 9; ++q) sPhi[vloc][k][q] = Phi[q];
        const float g0 = a.g[av], g1 = a.g[a.nV + av], g2 = a.g[2 * a.nV + av];
#pragma unroll
        for (int j = 0; j < 3; ++j) b[j] += Phi[j] * g0 + Phi[3 + j] * g1 + Phi[6 + j] * g2;
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
        dispgrad(a.u, a.nV, T, H);
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
            dispgrad(a.u, a.nV, T, H);
            kinematics(H, K, cH);
            float Phi[4][9];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int av = T.id[c];
                float U[9], Ra[9], T9[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) U[q] = rec[(5 + 9 * c + q) * a.S + s];
#pragma unroll
                for (int q = 0; q < 9; ++q) Ra[q] = a.R[q * a.nV + av];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj)
                        T9[3 * i + jj] = U[3 * i] * Ri[3 * jj] + U[3 * i + 1] * Ri[3 * jj + 1] + U[3 * i + 2] * Ri[3 * jj + 2];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj)
                        Phi[c][3 * i + jj] = Ra[3 * i] * T9[jj] + Ra[3 * i + 1] * T9[3 + jj] + Ra[3 * i + 2] * T9[6 + jj];
                const float gc = rec[(1 + c) * a.S + s];
                if (gc != 0.0f) {
                    const float g0 = a.g[av], g1 = a.g[a.nV + av], g2 = a.g[2 * a.nV + av];
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj)
                        b[jj] += gc * (Phi[c][jj] * g0 + Phi[c][3 + jj] * g1 + Phi[c][6 + jj] * g2);
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
        float gv[3] = {0.f, 0.f, 0.f};
        barrier_terms(a, v, gv, A6);  // barrier Hessian of vertex i only (gv unused: g holds it)
        float A[9] = {A6[0], A6[1], A6[2], A6[1], A6[3], A6[4], A6[2], A6[4], A6[5]};
        float bb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) bb[i] = b[i] + a.g[i * a.nV + v];
        float dx[3];
        local_solve(A, bb, dx);
#pragma unroll
        for (int i = 0; i < 3; ++i) a.unext[i * a.nV + v] = a.u[i * a.nV + v] + a.omega * dx[i];
    }
}

// ---------------------------------------------------------------------------
// Plain variant, one fused pass: g_i and H_ii from the incident tets, then
// x_i <- x_i - omega H_ii^-1 g_i.  Also leaves per-block |g|^2 partials of
// the iterate it read.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_plain(SweepArgs a) {
    const int lane = threadIdx.x % LPV;
    const int vloc = threadIdx.x / LPV;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int idx = blk * VPB + vloc;
    const int nidx = a.list ? a.n_list : a.nVf;
    const bool active = idx < nidx;
    const int f = active ? (a.list ? a.list[idx] : idx) : 0;
    float g[3] = {0.f, 0.f, 0.f}, A6[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (active) {
        const int n = a.inc_n[f];
        for (int j = lane; j < n; j += LPV) {
            const int pk = a.inc[(size_t)f * a.maxi + j];
            const int c = pk & 3;
            Tet T;
            load_tet(a.tet, pk >> 2, T);
            float H[9], cH[9], P[9], gn[3];
            Kin<float> K;
            dispgrad(a.u, a.nV, T, H);
            kinematics(H, K, cH);
            snh_stress_H(H, K, cH, T.vmu, T.vlam, P);
            gradN(T.D, c, gn);
#pragma unroll
            for (int i = 0; i < 3; ++i) g[i] += P[3 * i] * gn[0] + P[3 * i + 1] * gn[1] + P[3 * i + 2] * gn[2];
            int k = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float dF[9], dP[9];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int jj = 0; jj < 3; ++jj) dF[3 * i + jj] = (i == d) ? gn[jj] : 0.0f;
                snh_dstress(K.F, K.C, 1.0f + K.Jm1, T.vmu, T.vlam, dF, dP);
#pragma unroll
                for (int e = d; e < 3; ++e)
                    A6[k++] += dP[3 * e] * gn[0] + dP[3 * e + 1] * gn[1] + dP[3 * e + 2] * gn[2];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = lane_sum(g[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) A6[i] = lane_sum(A6[i]);
    double gsq = 0.0;
    if (active && lane == 0) {
        const int v = a.free_ids[f];
        const float m = a.mh2[v];
#pragma unroll
        for (int i = 0; i < 3; ++i) g[i] += m * (a.u[i * a.nV + v] - a.zu[i * a.nV + v]);
        A6[0] += m; A6[3] += m; A6[5] += m;
        barrier_terms(a, v, g, A6);
        gsq = (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
        float A[9] = {A6[0], A6[1], A6[2], A6[1], A6[3], A6[4], A6[2], A6[4], A6[5]};
        float dx[3];
        local_solve(A, g, dx);
        float* out = a.in_place ? const_cast<float*>(a.u) : a.unext;
        float un[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) un[i] = a.u[i * a.nV + v] + a.omega * dx[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) out[i * a.nV + v] = un[i];
    }
    block_partial(gsq, active && lane == 0, a.partial);
}

// Copies updated positions of the listed vertices from unext into u.
__global__ void k_commit(SweepArgs a) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n_list) return;
    const int v = a.free_ids[a.list[idx]];
#pragma unroll
    for (int i = 0; i < 3; ++i) const_cast<float*>(a.u)[i * a.nV + v] = a.unext[i * a.nV + v];
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

// z = xhat + h vhat + h^2 g on free vertices (displacement form), x0 = xhat.
__global__ void k_predict(int nV, const float* __restrict__ uhat, const float* __restrict__ vhat,
                          const float* __restrict__ mh2, float h, float g0, float g1, float g2,
                          float* __restrict__ u, float* __restrict__ unext, float* __restrict__ zu) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
    const float gg[3] = {g0, g1, g2};
    const bool free = mh2[v] > 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float x = uhat[i * nV + v];
        u[i * nV + v] = x;
        unext[i * nV + v] = x;
        zu[i * nV + v] = free ? x + h * vhat[i * nV + v] + h * h * gg[i] : x;
    }
}

// v = (x - xhat) / h ; xhat <- x
__global__ void k_velocity(int nV, const float* __restrict__ u, float* __restrict__ uhat,
                           float* __restrict__ vhat, float inv_h) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nV) return;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float x = u[i * nV + v];
        vhat[i * nV + v] = (x - uhat[i * nV + v]) * inv_h;
        uhat[i * nV + v] = x;
    }
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
        dispgrad(a.u, a.nV, T, H);
        kinematics(H, K, cH);
        e += (double)snh_psi_H(H, K, cH, T.vmu, T.vlam);
    }
    if (i < a.nVf) {
        const int v = a.free_ids[i];
        double in = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double d = (double)a.u[k * a.nV + v] - (double)a.zu[k * a.nV + v];
            in += d * d;
        }
        e += 0.5 * (double)a.mh2[v] * in;
        const double x[3] = {(double)a.X[v] + a.u[v], (double)a.X[a.nV + v] + a.u[a.nV + v],
                             (double)a.X[2 * a.nV + v] + a.u[2 * a.nV + v]};
        for (int p = 0; p < a.n_planes; ++p) {
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

void launch_phase1(jgs2_solver* s, const SweepArgs& a, bool want_R) {
    const int nb = n_blocks_for(a);
    if (nb == 0) return;
    hipLaunchKernelGGL(k_phase1, dim3(nb), dim3(BLOCK), 0, s->stream, a, want_R ? 1 : 0);
}

void launch_phase2_cubature(jgs2_solver* s, const SweepArgs& a) {
    const int nb = n_blocks_for(a);
    if (nb == 0) return;
    hipLaunchKernelGGL(k_phase2_cubature, dim3(nb), dim3(BLOCK), 0, s->stream, a);
}

void launch_plain(jgs2_solver* s, const SweepArgs& a) {
    const int nb = n_blocks_for(a);
    if (nb == 0) return;
    hipLaunchKernelGGL(k_plain, dim3(nb), dim3(BLOCK), 0, s->stream, a);
}

void launch_commit(jgs2_solver* s, const SweepArgs& a) {
    if (a.n_list == 0) return;
    hipLaunchKernelGGL(k_commit, dim3((a.n_list + 255) / 256), dim3(256), 0, s->stream, a);
}

void launch_reduce(jgs2_solver* s, int n) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s->stream, s->d_partial, n, s->d_red);
}

void launch_predict(jgs2_solver* s, float h, const float* grav) {
    hipLaunchKernelGGL(k_predict, dim3((s->nV + 255) / 256), dim3(256), 0, s->stream, s->nV, s->d_uhat,
                       s->d_vhat, s->d_mh2, h, grav[0], grav[1], grav[2], s->d_u, s->d_unext, s->d_zu);
}

void launch_velocity(jgs2_solver* s, float h) {
    hipLaunchKernelGGL(k_velocity, dim3((s->nV + 255) / 256), dim3(256), 0, s->stream, s->nV, s->d_u, s->d_uhat,
                       s->d_vhat, 1.0f / h);
}

void launch_energy(jgs2_solver* s, const SweepArgs& a, int nT) {
    const int n = nT > a.nVf ? nT : a.nVf;
    hipLaunchKernelGGL(k_energy, dim3((n + 255) / 256), dim3(256), 0, s->stream, a, nT);
}

}  // namespace jgs2
