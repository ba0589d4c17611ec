// Device-side building blocks of the fused ALE Galerkin-Boltzmann stage kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gbd {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt2 = 1.41421356237309504880;

// Prescribed vertex motion (mirrors gb_motion of the C interface).
struct Motion {
    int kind;
    double p[8];
    // kind 4 (vertex array): velocities of every vertex at the four stage
    // times t_n, t_n + dt/2, t_n + dt/2, t_n + dt, [4][nv][DIM], device memory
    const double *w;
};

// Grid velocity v_G(X, t) = d/dt of the prescribed displacement at fixed
// reference position X (Section 5; motion formulas of Sections 7.1-7.4).
template <int DIM>
__device__ __forceinline__ void motion_velocity(const Motion &m, const double *X, double t, double *w) {
    for (int d = 0; d < DIM; ++d) w[d] = 0.0;
    if (m.kind == 1) {  // sin product (eq. gcl_exact_field)
        const double om = 2.0 * kPi / m.p[2];
        const double tt = om * cos(om * t);
        const double sp = sin(2.0 * kPi * (X[0] - m.p[5]) / m.p[3]) * sin(2.0 * kPi * (X[1] - m.p[6]) / m.p[4]);
        w[0] = m.p[0] * tt * sp;
        w[1] = m.p[1] * tt * sp;
    } else if (m.kind == 2) {  // triple product (eq. TGV_deformation)
        if constexpr (DIM == 3) {
            const double om = 2.0 * kPi / m.p[1];
            const double tt = om * cos(om * t);
            const double L = m.p[2];
            double s[3];
            for (int d = 0; d < 3; ++d) s[d] = sin(2.0 * kPi * (X[d] + 0.5 * L) / L);
            w[0] = m.p[0] * tt * s[1] * s[2];
            w[1] = m.p[0] * tt * s[0] * s[2];
            w[2] = m.p[0] * tt * s[0] * s[1];
        }
    } else if (m.kind == 3) {  // plunge with radial blend
        const double om = m.p[1];
        const double tt = om * cos(om * t);
        const double dx = X[0] - m.p[4], dy = X[1] - m.p[5];
        const double r = sqrt(dx * dx + dy * dy);
        double xi = (r - m.p[2]) / (m.p[3] - m.p[2]);
        xi = xi < 0.0 ? 0.0 : (xi > 1.0 ? 1.0 : xi);
        const double B = 0.5 * (1.0 + cos(kPi * xi));
        w[1] = -m.p[0] * tt * B;
    } else if (m.kind == 5) {  // carangiform swimming (Section 7.4), z only
        if constexpr (DIM == 3) {
            const double xt = X[0] < 0.0 ? 0.0 : (X[0] > 1.0 ? 1.0 : X[0]);
            const double amp = m.p[0] + m.p[1] * xt + m.p[2] * xt * xt;
            const double om = 2.0 * kPi * m.p[4];
            const double phi = 2.0 * kPi * X[0] / m.p[3] - om * t;
            const double dx = X[0] - xt;
            double dist = sqrt(dx * dx + X[1] * X[1] + X[2] * X[2]) - m.p[5];
            dist = dist > 0.0 ? dist : 0.0;
            const double B = exp(-m.p[6] * dist * dist);
            double S = 1.0, dS = 0.0;
            if (m.p[7] > 0.0 && t < m.p[7]) {
                const double a = kPi / m.p[7];
                S = 0.5 * (1.0 - cos(a * t));
                dS = 0.5 * a * sin(a * t);
            }
            w[2] = amp * B * (-om * cos(phi) * S + sin(phi) * dS);
        }
    }
}

// y = M_n x for the normal-flux pattern M_n = sum_d n_d M_d of the moment
// system (A_d = -c M_d; Section 2 for 2D, tensor form for 3D).
template <int DIM, typename T>
__device__ __forceinline__ void apply_Mn(const T *n, const T *x, T *y) {
    const T s2 = T(kSqrt2);
    if constexpr (DIM == 2) {
        const T nx = n[0], ny = n[1];
        y[0] = nx * x[1] + ny * x[2];
        y[1] = nx * (x[0] + s2 * x[4]) + ny * x[3];
        y[2] = nx * x[3] + ny * (x[0] + s2 * x[5]);
        y[3] = nx * x[2] + ny * x[1];
        y[4] = s2 * nx * x[1];
        y[5] = s2 * ny * x[2];
    } else {
        // fields: rho, mx, my, mz, Sxy, Sxz, Syz, qxx, qyy, qzz (q_ii = S_ii/sqrt2)
        const T nx = n[0], ny = n[1], nz = n[2];
        y[0] = nx * x[1] + ny * x[2] + nz * x[3];
        y[1] = nx * (x[0] + s2 * x[7]) + ny * x[4] + nz * x[5];
        y[2] = nx * x[4] + ny * (x[0] + s2 * x[8]) + nz * x[6];
        y[3] = nx * x[5] + ny * x[6] + nz * (x[0] + s2 * x[9]);
        y[4] = nx * x[2] + ny * x[1];
        y[5] = nx * x[3] + nz * x[1];
        y[6] = ny * x[3] + nz * x[2];
        y[7] = s2 * nx * x[1];
        y[8] = s2 * ny * x[2];
        y[9] = s2 * nz * x[3];
    }
}

// Volume operator contribution for one gradient direction d:
// out -= c * (M_d g)   (A_d . grad q with A_d = -c M_d).
template <int DIM, int D, typename T>
__device__ __forceinline__ void sub_cMd(T c, const T *g, T *out) {
    const T s2 = T(kSqrt2);
    if constexpr (DIM == 2) {
        if constexpr (D == 0) {
            out[0] -= c * g[1];
            out[1] -= c * (g[0] + s2 * g[4]);
            out[2] -= c * g[3];
            out[3] -= c * g[2];
            out[4] -= c * s2 * g[1];
        } else {
            out[0] -= c * g[2];
            out[1] -= c * g[3];
            out[2] -= c * (g[0] + s2 * g[5]);
            out[3] -= c * g[1];
            out[5] -= c * s2 * g[2];
        }
    } else {
        if constexpr (D == 0) {
            out[0] -= c * g[1];
            out[1] -= c * (g[0] + s2 * g[7]);
            out[2] -= c * g[4];
            out[3] -= c * g[5];
            out[4] -= c * g[2];
            out[5] -= c * g[3];
            out[7] -= c * s2 * g[1];
        } else if constexpr (D == 1) {
            out[0] -= c * g[2];
            out[1] -= c * g[4];
            out[2] -= c * (g[0] + s2 * g[8]);
            out[3] -= c * g[6];
            out[4] -= c * g[1];
            out[6] -= c * g[3];
            out[8] -= c * s2 * g[2];
        } else {
            out[0] -= c * g[3];
            out[1] -= c * g[5];
            out[2] -= c * g[6];
            out[3] -= c * (g[0] + s2 * g[9]);
            out[5] -= c * g[1];
            out[6] -= c * g[2];
            out[9] -= c * s2 * g[3];
        }
    }
}

// Reciprocal and reciprocal square root from the hardware approximations
// (v_rcp / v_rsq) refined by Newton-Raphson steps: one step in FP32 (the
// approximation is within 1 ulp), two in FP64 (each step doubles the correct
// bits of the approximation); a handful of instructions instead of the
// correctly rounded division and square root sequences.
__device__ __forceinline__ float rcp_nr(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
    const double h = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return fma(y, fma(-h * y, y, 0.5), y);
}
// The same, refined only as far as a result that is cast to T needs: one
// Newton step (relative error about 2^-44) when T is FP32, two for FP64.
template <typename T>
__device__ __forceinline__ double rcp_for(double x) {
    if constexpr (sizeof(T) == 8) return rcp_nr(x);
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
template <typename T>
__device__ __forceinline__ double rsq_for(double x) {
    if constexpr (sizeof(T) == 8) return rsq_nr(x);
    const double y = __builtin_amdgcn_rsq(x);
    return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}

// Nonlinear relaxation source Ntilde (Section 4) for the stress fields,
// given density and momentum at a point: m_a m_b / (tau rho) off the
// diagonal, m_a^2 / (sqrt2 tau rho) on it.
template <int DIM, typename T>
__device__ __forceinline__ void ntilde(T rho, const T *m, T inv_tau, T *out) {
    const T k = inv_tau * rcp_nr(rho);
    const T kd = k * T(1.0 / kSqrt2);
    if constexpr (DIM == 2) {
        out[0] = k * m[0] * m[1];
        out[1] = kd * m[0] * m[0];
        out[2] = kd * m[1] * m[1];
    } else {
        out[0] = k * m[0] * m[1];
        out[1] = k * m[0] * m[2];
        out[2] = k * m[1] * m[2];
        out[3] = kd * m[0] * m[0];
        out[4] = kd * m[1] * m[1];
        out[5] = kd * m[2] * m[2];
    }
}

}  // namespace gbd
