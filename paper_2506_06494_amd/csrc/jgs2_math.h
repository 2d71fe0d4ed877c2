// Small dense math for the JGS2 kernels (device and host), templated on the
// scalar type: float in the sweeps, double in the precompute.
//
// Material: stable Neo-Hookean (Sec. 8 / Table 1 caption); the energy used
// is Psi = mu/2 (|F|^2 - 3) - mu (J - 1) + lam/2 (J - 1)^2 with
// mu = mu_L, lam = lam_L + mu_L, which linearises to linear elasticity with
// the given (E, nu).  Quantities named v* are pre-multiplied by the tet
// volume.
#pragma once
#include <hip/hip_runtime.h>

#define JGS2_HD __host__ __device__ __forceinline__

namespace jgs2 {

template <typename T> struct M3 { T a[9]; };  // row-major 3x3

template <typename T> JGS2_HD T det3(const T* F) {
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

// cof(F): column k is the cross product of the other two columns of F
// (cyclically), so cof(F) = det(F) F^-T.
template <typename T> JGS2_HD void cof3(const T* F, T* C) {
    C[0] = F[4] * F[8] - F[7] * F[5];
    C[3] = F[7] * F[2] - F[1] * F[8];
    C[6] = F[1] * F[5] - F[4] * F[2];
    C[1] = F[5] * F[6] - F[8] * F[3];
    C[4] = F[8] * F[0] - F[2] * F[6];
    C[7] = F[2] * F[3] - F[5] * F[0];
    C[2] = F[3] * F[7] - F[6] * F[4];
    C[5] = F[6] * F[1] - F[0] * F[7];
    C[8] = F[0] * F[4] - F[3] * F[1];
}

// Directional derivative of cof at F along D.
template <typename T> JGS2_HD void dcof3(const T* F, const T* D, T* C) {
    C[0] = D[4] * F[8] + F[4] * D[8] - D[7] * F[5] - F[7] * D[5];
    C[3] = D[7] * F[2] + F[7] * D[2] - D[1] * F[8] - F[1] * D[8];
    C[6] = D[1] * F[5] + F[1] * D[5] - D[4] * F[2] - F[4] * D[2];
    C[1] = D[5] * F[6] + F[5] * D[6] - D[8] * F[3] - F[8] * D[3];
    C[4] = D[8] * F[0] + F[8] * D[0] - D[2] * F[6] - F[2] * D[6];
    C[7] = D[2] * F[3] + F[2] * D[3] - D[5] * F[0] - F[5] * D[0];
    C[2] = D[3] * F[7] + F[3] * D[7] - D[6] * F[4] - F[6] * D[4];
    C[5] = D[6] * F[1] + F[6] * D[1] - D[0] * F[7] - F[0] * D[7];
    C[8] = D[0] * F[4] + F[0] * D[4] - D[3] * F[1] - F[3] * D[1];
}

// Volume-scaled first Piola-Kirchhoff stress V P(F).
template <typename T> JGS2_HD void snh_stress(const T* F, const T* C, T J, T vmu, T vlam, T* P) {
    const T k = vlam * (J - T(1)) - vmu;
#pragma unroll
    for (int i = 0; i < 9; ++i) P[i] = vmu * F[i] + k * C[i];
}

// Volume-scaled stress differential V dP[D].
template <typename T> JGS2_HD void snh_dstress(const T* F, const T* C, T J, T vmu, T vlam,
                                               const T* D, T* dP) {
    T CD = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) CD += C[i] * D[i];
    T dC[9];
    dcof3(F, D, dC);
    const T k = vlam * (J - T(1)) - vmu;
    const T l = vlam * CD;
#pragma unroll
    for (int i = 0; i < 9; ++i) dP[i] = vmu * D[i] + l * C[i] + k * dC[i];
}

// The same quantities from the displacement gradient H = F - I without the
// O(mu) cancellation of F - cof F at small strain (needed in FP32):
//   cof(I + H) = I + tr(H) I - H^T + cof(H)
//   J - 1      = tr(H) + tr(cof H) + det(H)
//   V P        = V mu (H + H^T - tr(H) I - cof H) + V lam (J - 1) cof(F)
//   V Psi      = V mu/2 |H|^2 - V mu (tr(cof H) + det H) + V lam/2 (J - 1)^2
template <typename T> struct Kin {
    T F[9], C[9];  // F = I + H and cof F
    T Jm1;         // J - 1
};

template <typename T> JGS2_HD void kinematics(const T* H, Kin<T>& k, T* cofH) {
    cof3(H, cofH);
    const T trH = H[0] + H[4] + H[8];
    const T i2 = cofH[0] + cofH[4] + cofH[8];
    k.Jm1 = trH + i2 + det3(H);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T d = (i == j) ? T(1) : T(0);
            k.F[3 * i + j] = d + H[3 * i + j];
            k.C[3 * i + j] = d + d * trH - H[3 * j + i] + cofH[3 * i + j];
        }
}

template <typename T> JGS2_HD void snh_stress_H(const T* H, const Kin<T>& k, const T* cofH, T vmu, T vlam, T* P) {
    const T trH = H[0] + H[4] + H[8];
    const T l = vlam * k.Jm1;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T d = (i == j) ? trH : T(0);
            P[3 * i + j] = vmu * (H[3 * i + j] + H[3 * j + i] - d - cofH[3 * i + j]) + l * k.C[3 * i + j];
        }
}

template <typename T> JGS2_HD T snh_psi_H(const T* H, const Kin<T>& k, const T* cofH, T vmu, T vlam) {
    T H2 = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) H2 += H[i] * H[i];
    const T i2 = cofH[0] + cofH[4] + cofH[8];
    return T(0.5) * vmu * H2 - vmu * (i2 + det3(H)) + T(0.5) * vlam * k.Jm1 * k.Jm1;
}

template <typename T> JGS2_HD T snh_psi(const T* F, T J, T vmu, T vlam) {
    T I2 = T(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) I2 += F[i] * F[i];
    return T(0.5) * vmu * (I2 - T(3)) - vmu * (J - T(1)) + T(0.5) * vlam * (J - T(1)) * (J - T(1));
}

// IPC log barrier B(d) = -(d - dh)^2 log(d / dh) on 0 < d < dh (Eq. barrier)
// and its first two derivatives.
template <typename T> JGS2_HD T barrier(T d, T dh) {
    if (d >= dh) return T(0);
    return -(d - dh) * (d - dh) * log(d / dh);
}
template <typename T> JGS2_HD T barrier_d1(T d, T dh) {
    if (d >= dh) return T(0);
    return -T(2) * (d - dh) * log(d / dh) - (d - dh) * (d - dh) / d;
}
template <typename T> JGS2_HD T barrier_d2(T d, T dh) {
    if (d >= dh) return T(0);
    const T r = (d - dh) / d;
    return -T(2) * log(d / dh) - T(4) * r + r * r;
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations.
// A (row-major, symmetric) is overwritten; w receives the eigenvalues and
// V (row-major) the eigenvectors as columns.
template <typename T> JGS2_HD void sym_eig3(T* A, T* w, T* V) {
#pragma unroll
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? T(1) : T(0);
    for (int sweep = 0; sweep < 8; ++sweep) {
        const T off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const T dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= dia * T(1e-30) || off == T(0)) break;
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0;
            const int q = pq == 0 ? 1 : 2;
            const T apq = A[3 * p + q];
            if (apq == T(0)) continue;
            const T theta = (A[3 * q + q] - A[3 * p + p]) / (T(2) * apq);
            const T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
            const T c = T(1) / sqrt(t * t + T(1));
            const T s = t * c;
            // A <- G^T A G with G the (p,q) rotation
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T akp = A[3 * k + p], akq = A[3 * k + q];
                A[3 * k + p] = c * akp - s * akq;
                A[3 * k + q] = s * akp + c * akq;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T apk = A[3 * p + k], aqk = A[3 * q + k];
                A[3 * p + k] = c * apk - s * aqk;
                A[3 * q + k] = s * apk + c * aqk;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T vkp = V[3 * k + p], vkq = V[3 * k + q];
                V[3 * k + p] = c * vkp - s * vkq;
                V[3 * k + q] = s * vkp + c * vkq;
            }
        }
    }
    w[0] = A[0]; w[1] = A[4]; w[2] = A[8];
}

// Closest rotation to F (the rotation of the polar decomposition when
// det F > 0; otherwise U diag(1,1,det(U V^T)) V^T of the SVD):
// with the eigenvectors v_k of F^T F, let a, b index the two largest
// eigenvalues and m the smallest; u_k = F v_k / sigma_k; then
// R = u_a v_a^T + u_b v_b^T + det[v_a v_b v_m] (u_a x u_b) v_m^T.
template <typename T> JGS2_HD void closest_rotation(const T* F, T* R) {
    T C[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
    T w[3], V[9];
    sym_eig3(C, w, V);
    // m = index of the smallest eigenvalue, (a, b) = the other two (static selects)
    const bool m0 = (w[0] <= w[1]) && (w[0] <= w[2]);
    const bool m1 = !m0 && (w[1] <= w[2]);
    T va[3], vb[3], vm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T c0 = V[3 * i], c1 = V[3 * i + 1], c2 = V[3 * i + 2];
        vm[i] = m0 ? c0 : (m1 ? c1 : c2);
        va[i] = m0 ? c1 : (m1 ? c2 : c0);
        vb[i] = m0 ? c2 : (m1 ? c0 : c1);
    }
    const T wa = m0 ? w[1] : (m1 ? w[2] : w[0]);
    const T wb = m0 ? w[2] : (m1 ? w[0] : w[1]);
    const T sa = sqrt(wa > T(0) ? wa : T(0));
    const T sb = sqrt(wb > T(0) ? wb : T(0));
    if (!(sa > T(0)) || !(sb > T(0))) {  // rank <= 1: no unique rotation
#pragma unroll
        for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? T(1) : T(0);
        return;
    }
    T ua[3], ub[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ua[i] = (F[3 * i] * va[0] + F[3 * i + 1] * va[1] + F[3 * i + 2] * va[2]) / sa;
        ub[i] = (F[3 * i] * vb[0] + F[3 * i + 1] * vb[1] + F[3 * i + 2] * vb[2]) / sb;
    }
    T um[3] = {ua[1] * ub[2] - ua[2] * ub[1], ua[2] * ub[0] - ua[0] * ub[2], ua[0] * ub[1] - ua[1] * ub[0]};
    const T dv = va[0] * (vb[1] * vm[2] - vb[2] * vm[1]) - va[1] * (vb[0] * vm[2] - vb[2] * vm[0]) +
                 va[2] * (vb[0] * vm[1] - vb[1] * vm[0]);
    const T sgn = dv >= T(0) ? T(1) : T(-1);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            R[3 * i + j] = ua[i] * va[j] + ub[i] * vb[j] + sgn * um[i] * vm[j];
}

// Rotation of the polar decomposition F = R S for det F > 0 by Higham's
// scaled Newton iteration X <- (zeta X + X^-T / zeta) / 2 with
// zeta = sqrt(|X^-1|_F / |X|_F), then one unscaled step once the update is
// below 1e-4 |X|.  Falls back to the eigen route (closest_rotation, which
// also covers det F <= 0).
template <typename T> JGS2_HD void polar_rotation(const T* F, T* R) {
    T X[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) X[i] = F[i];
    if (!(det3(X) > T(0))) {
        closest_rotation(F, R);
        return;
    }
    bool done = false;
    for (int it = 0; it < 24 && !done; ++it) {
        T C[9];
        cof3(X, C);
        const T det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
        T nX = T(0), nC = T(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) { nX += X[i] * X[i]; nC += C[i] * C[i]; }
        nX = sqrt(nX);
        nC = sqrt(nC);
        T zeta = sqrt((nC / det) / nX);
        T diff = T(0);
        for (int pass = 0; pass < 2; ++pass) {
            const T a = T(0.5) * zeta, b = T(0.5) / (zeta * det);
            T Xn[9];
            diff = T(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                Xn[i] = a * X[i] + b * C[i];
                diff += (Xn[i] - X[i]) * (Xn[i] - X[i]);
            }
            if (pass == 0) {
#pragma unroll
                for (int i = 0; i < 9; ++i) X[i] = Xn[i];
                if (diff > T(1e-8) * nX * nX) break;  // keep iterating with scaling
                // converged to ~1e-4: one unscaled polishing step
                cof3(X, C);
                const T d2 = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
                zeta = T(1);
                const T a2 = T(0.5), b2 = T(0.5) / d2;
#pragma unroll
                for (int i = 0; i < 9; ++i) X[i] = a2 * X[i] + b2 * C[i];
                done = true;
                break;
            }
        }
    }
    if (!done) {
        closest_rotation(F, R);
        return;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = X[i];
}

// Unit quaternion (x, y, z, w) of a rotation matrix (Shepperd's branches)
// and back.
template <typename T> JGS2_HD void quat_from_rot(const T* R, T* q) {
    const T tr = R[0] + R[4] + R[8];
    T x, y, z, w;
    if (tr > T(0)) {
        const T s = sqrt(tr + T(1)) * T(2);
        w = T(0.25) * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
    } else if (R[0] > R[4] && R[0] > R[8]) {
        const T s = sqrt(T(1) + R[0] - R[4] - R[8]) * T(2);
        w = (R[7] - R[5]) / s; x = T(0.25) * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
    } else if (R[4] > R[8]) {
        const T s = sqrt(T(1) + R[4] - R[0] - R[8]) * T(2);
        w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = T(0.25) * s; z = (R[5] + R[7]) / s;
    } else {
        const T s = sqrt(T(1) + R[8] - R[0] - R[4]) * T(2);
        w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = T(0.25) * s;
    }
    const T n = T(1) / sqrt(x * x + y * y + z * z + w * w);
    q[0] = x * n; q[1] = y * n; q[2] = z * n; q[3] = w * n;
}

template <typename T> JGS2_HD void rot_from_quat(T x, T y, T z, T w, T* R) {
    R[0] = T(1) - T(2) * (y * y + z * z); R[1] = T(2) * (x * y - z * w); R[2] = T(2) * (x * z + y * w);
    R[3] = T(2) * (x * y + z * w); R[4] = T(1) - T(2) * (x * x + z * z); R[5] = T(2) * (y * z - x * w);
    R[6] = T(2) * (x * z - y * w); R[7] = T(2) * (y * z + x * w); R[8] = T(1) - T(2) * (x * x + y * y);
}

// Reciprocal: v_rcp_f32 (within 1 ulp) for float, exact division for double.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// LDL^T pivots of a symmetric 3x3 (lower triangle used) and their
// reciprocals (a zero pivot has a zero multiplier column).
template <typename T> __device__ __forceinline__ void ldl_pivots(const T* A, T* d, T* inv, T* l10, T* l20, T* l21) {
    d[0] = A[0];
    inv[0] = recip(d[0]);
    const T i0 = d[0] != T(0) ? inv[0] : T(0);
    *l10 = A[3] * i0;
    *l20 = A[6] * i0;
    d[1] = A[4] - (*l10) * (*l10) * d[0];
    inv[1] = recip(d[1]);
    *l21 = d[1] != T(0) ? (A[7] - (*l20) * (*l10) * d[0]) * inv[1] : T(0);
    d[2] = A[8] - (*l20) * (*l20) * d[0] - (*l21) * (*l21) * d[1];
    inv[2] = recip(d[2]);
}

// dx = -A^-1 b for a symmetric 3x3 A.  If A is not safely positive definite
// (an LDL^T pivot <= 1e-6 |tr A|), A is shifted by (|d_min| + 1e-6 |tr A|) I,
// the shift doubling until it is.
template <typename T> __device__ __forceinline__ void local_solve(const T* A_in, const T* b, T* dx) {
    T A[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) A[i] = A_in[i];
    const T tr = fabs(A[0] + A[4] + A[8]);
    T d[3], inv[3], l10, l20, l21;
    ldl_pivots(A, d, inv, &l10, &l20, &l21);
    T dmin = fmin(d[0], fmin(d[1], d[2]));
    if (!(dmin > T(1e-6) * tr)) {
        T shift = fabs(dmin) + T(1e-6) * tr;
        for (int it = 0; it < 60; ++it) {
            T As[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) As[i] = A[i];
            As[0] += shift; As[4] += shift; As[8] += shift;
            ldl_pivots(As, d, inv, &l10, &l20, &l21);
            dmin = fmin(d[0], fmin(d[1], d[2]));
            if (dmin > T(1e-6) * tr) break;
            shift *= T(2);
        }
    }
    // forward: L y = b ; diagonal ; back: L^T x = y
    T y0 = b[0];
    T y1 = b[1] - l10 * y0;
    T y2 = b[2] - l20 * y0 - l21 * y1;
    y0 *= inv[0]; y1 *= inv[1]; y2 *= inv[2];
    T x2 = y2;
    T x1 = y1 - l21 * x2;
    T x0 = y0 - l10 * x1 - l20 * x2;
    dx[0] = -x0; dx[1] = -x1; dx[2] = -x2;
}

}  // namespace jgs2
