// Flow diagnostics and state setup kernels (outside the stepping path):
//   * kinetic energy of Section 7.2 and its exact rate along the
//     semi-discrete system (epsilon_1 = -dE_K/dt), as a two-pass FP64
//     reduction over elements;
//   * pressure and viscous force on the wall faces (the c_D / c_L
//     integrals of Section 7.3, split as in Section 7.4);
//   * the equilibrium map of Section 2 from density and velocity to moments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gb_device.hpp"

namespace gbd {

constexpr int kDiagBlock = 256;           // threads per workgroup of the reduction kernels
constexpr int kDiagSums = 4;              // integral, its rate, volume, its rate

// Element-wise data the energy kernel reads: the state Q and its right-hand
// side F (blocked [K/16][NF][Np][16] in the storage type T), the vertex
// positions and grid velocities of the current time, the cubature rule.
template <typename T>
struct EnergyArgs {
    int64_t K;
    int Np, NF, Nc, dim;
    const T *Q, *F;
    const int32_t *etov;
    const double *x, *w;       // [nv][dim]
    const double *Icub;        // [Nc][Np]
    const double *wcub;        // [Nc]
    double c, rho0;
    double *partial;           // [gridDim.x][kDiagSums]
};

// Sum of v over the workgroup in a fixed order (tree over LDS), result in
// lane 0 of wave 0; every thread must call it.
__device__ inline double block_sum(double v, double *s_red) {
    s_red[threadIdx.x] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) s_red[threadIdx.x] += s_red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = s_red[0];
    __syncthreads();
    return r;
}

// One wavefront per element (grid-stride), lanes over the cubature points.
// Per element: I_e = J sum_c w_c e_c with e = c^2 |m|^2 / (2 rho), its rate
// J div(w) sum_c w_c e_c + J sum_c w_c (de/drho rhodot + de/dm . mdot), and
// the volume J sum_c w_c with its rate J div(w) sum_c w_c.
template <int DIM, typename T>
__global__ void __launch_bounds__(kDiagBlock) energy_partial_kernel(EnergyArgs<T> a) {
    constexpr int NC = DIM + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    double *s_I = reinterpret_cast<double *>(smem);            // [Nc][Np]
    double *s_w = s_I + a.Nc * a.Np;                           // [Nc]
    double *s_red = s_w + a.Nc;                                // [blockDim]
    double *s_q = s_red + blockDim.x;                          // per wave [2][NC][Np]
    for (int p = threadIdx.x; p < a.Nc * a.Np; p += blockDim.x) s_I[p] = a.Icub[p];
    for (int p = threadIdx.x; p < a.Nc; p += blockDim.x) s_w[p] = a.wcub[p];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    double *q = s_q + wave * 2 * NC * a.Np;
    double *f = q + NC * a.Np;
    double acc[kDiagSums] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = int64_t(gridDim.x) * waves;
    for (int64_t e = int64_t(blockIdx.x) * waves + wave; e < a.K; e += stride) {
        // density and momentum of the element and their right-hand side
        for (int p = lane; p < NC * a.Np; p += 64) {
            const int k = p / a.Np, j = p - k * a.Np;
            const int64_t off = (((e >> 4) * a.NF + k) * a.Np + j) * 16 + (e & 15);
            q[p] = double(a.Q[off]) + (k == 0 ? a.rho0 : 0.0);
            f[p] = double(a.F[off]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // affine map: J and dr/dx, and div(w) of the linear grid velocity
        double xv[DIM + 1][DIM], wv[DIM + 1][DIM];
        for (int v = 0; v <= DIM; ++v) {
            const int64_t gv = a.etov[e * (DIM + 1) + v];
            for (int d = 0; d < DIM; ++d) {
                xv[v][d] = a.x[gv * DIM + d];
                wv[v][d] = a.w[gv * DIM + d];
            }
        }
        double G[DIM][DIM], Wr[DIM][DIM];   // G[i][a] = dx_i/dr_a, Wr[i][a] = dw_i/dr_a
        for (int i = 0; i < DIM; ++i)
            for (int aa = 0; aa < DIM; ++aa) {
                G[i][aa] = 0.5 * (xv[aa + 1][i] - xv[0][i]);
                Wr[i][aa] = 0.5 * (wv[aa + 1][i] - wv[0][i]);
            }
        double J, divw = 0.0;
        if constexpr (DIM == 2) {
            J = G[0][0] * G[1][1] - G[0][1] * G[1][0];
            // div w = trace(Wr G^-1), G^-1 = adj(G) / J
            divw = (Wr[0][0] * G[1][1] - Wr[0][1] * G[1][0] - Wr[1][0] * G[0][1] + Wr[1][1] * G[0][0]) / J;
        } else {
            double C[3][3];   // cofactors: (G^-1)[a][i] = C[i][a] / J
            for (int i = 0; i < 3; ++i)
                for (int aa = 0; aa < 3; ++aa) {
                    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, a1 = (aa + 1) % 3, a2 = (aa + 2) % 3;
                    C[i][aa] = G[i1][a1] * G[i2][a2] - G[i1][a2] * G[i2][a1];
                }
            J = G[0][0] * C[0][0] + G[0][1] * C[0][1] + G[0][2] * C[0][2];
            for (int i = 0; i < 3; ++i)
                for (int aa = 0; aa < 3; ++aa) divw += Wr[i][aa] * C[i][aa];
            divw /= J;
        }
        const double c2 = a.c * a.c;
        double se = 0.0, sde = 0.0, sw = 0.0;
        for (int p = lane; p < a.Nc; p += 64) {
            const double *Ir = s_I + p * a.Np;
            double v[NC], dv[NC];
            for (int k = 0; k < NC; ++k) {
                double s0 = 0.0, s1 = 0.0;
                for (int j = 0; j < a.Np; ++j) {
                    s0 += Ir[j] * q[k * a.Np + j];
                    s1 += Ir[j] * f[k * a.Np + j];
                }
                v[k] = s0;
                dv[k] = s1;
            }
            double mm = 0.0, mdm = 0.0;
            for (int d = 0; d < DIM; ++d) {
                mm += v[1 + d] * v[1 + d];
                mdm += v[1 + d] * dv[1 + d];
            }
            const double ir = 1.0 / v[0];
            const double e_c = 0.5 * c2 * mm * ir;
            const double de_c = c2 * mdm * ir - 0.5 * c2 * mm * dv[0] * ir * ir;
            se += s_w[p] * e_c;
            sde += s_w[p] * de_c;
            sw += s_w[p];
        }
        acc[0] += J * se;
        acc[1] += J * divw * se + J * sde;
        acc[2] += J * sw;
        acc[3] += J * divw * sw;
        __builtin_amdgcn_wave_barrier();    // q, f reused by the wave's next element
    }
    for (int k = 0; k < kDiagSums; ++k) {
        const double s = block_sum(acc[k], s_red);
        if (threadIdx.x == 0) a.partial[int64_t(blockIdx.x) * kDiagSums + k] = s;
    }
}

// The same sums (same per-lane order of points and terms) with the
// interpolation rows of the lane's two cubature points (p = lane and
// lane + 64, so Nc <= 128) held in registers for the whole launch instead of
// read from LDS for every element; the order's node count NP is a template
// parameter so that the rows stay in registers.
template <int DIM, typename T, int NP>
__global__ void __launch_bounds__(kDiagBlock) energy_partial_reg_kernel(EnergyArgs<T> a) {
    constexpr int NC = DIM + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    double *s_red = reinterpret_cast<double *>(smem);         // [blockDim]
    double *s_q = s_red + blockDim.x;                          // per wave [2][NC][NP]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    double *q = s_q + wave * 2 * NC * NP;
    double *f = q + NC * NP;
    double Ir[2][NP], wc[2];
    bool live[2];
#pragma unroll
    for (int pt = 0; pt < 2; ++pt) {
        const int p = lane + 64 * pt;
        live[pt] = p < a.Nc;
        const int pc = live[pt] ? p : 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) Ir[pt][j] = a.Icub[pc * NP + j];
        wc[pt] = a.wcub[pc];
    }
    double acc[kDiagSums] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = int64_t(gridDim.x) * waves;
    for (int64_t e = int64_t(blockIdx.x) * waves + wave; e < a.K; e += stride) {
        for (int p = lane; p < NC * NP; p += 64) {
            const int k = p / NP, j = p - k * NP;
            const int64_t off = (((e >> 4) * a.NF + k) * NP + j) * 16 + (e & 15);
            q[p] = double(a.Q[off]) + (k == 0 ? a.rho0 : 0.0);
            f[p] = double(a.F[off]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double xv[DIM + 1][DIM], wv[DIM + 1][DIM];
        for (int v = 0; v <= DIM; ++v) {
            const int64_t gv = a.etov[e * (DIM + 1) + v];
            for (int d = 0; d < DIM; ++d) {
                xv[v][d] = a.x[gv * DIM + d];
                wv[v][d] = a.w[gv * DIM + d];
            }
        }
        double G[DIM][DIM], Wr[DIM][DIM];
        for (int i = 0; i < DIM; ++i)
            for (int aa = 0; aa < DIM; ++aa) {
                G[i][aa] = 0.5 * (xv[aa + 1][i] - xv[0][i]);
                Wr[i][aa] = 0.5 * (wv[aa + 1][i] - wv[0][i]);
            }
        double J, divw = 0.0;
        if constexpr (DIM == 2) {
            J = G[0][0] * G[1][1] - G[0][1] * G[1][0];
            divw = (Wr[0][0] * G[1][1] - Wr[0][1] * G[1][0] - Wr[1][0] * G[0][1] + Wr[1][1] * G[0][0]) / J;
        } else {
            double C[3][3];
            for (int i = 0; i < 3; ++i)
                for (int aa = 0; aa < 3; ++aa) {
                    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, a1 = (aa + 1) % 3, a2 = (aa + 2) % 3;
                    C[i][aa] = G[i1][a1] * G[i2][a2] - G[i1][a2] * G[i2][a1];
                }
            J = G[0][0] * C[0][0] + G[0][1] * C[0][1] + G[0][2] * C[0][2];
            for (int i = 0; i < 3; ++i)
                for (int aa = 0; aa < 3; ++aa) divw += Wr[i][aa] * C[i][aa];
            divw /= J;
        }
        const double c2 = a.c * a.c;
        double se = 0.0, sde = 0.0, sw = 0.0;
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
            if (!live[pt]) continue;
            double v[NC], dv[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    s0 += Ir[pt][j] * q[k * NP + j];
                    s1 += Ir[pt][j] * f[k * NP + j];
                }
                v[k] = s0;
                dv[k] = s1;
            }
            double mm = 0.0, mdm = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                mm += v[1 + d] * v[1 + d];
                mdm += v[1 + d] * dv[1 + d];
            }
            const double ir = 1.0 / v[0];
            const double e_c = 0.5 * c2 * mm * ir;
            const double de_c = c2 * mdm * ir - 0.5 * c2 * mm * dv[0] * ir * ir;
            se += wc[pt] * e_c;
            sde += wc[pt] * de_c;
            sw += wc[pt];
        }
        acc[0] += J * se;
        acc[1] += J * divw * se + J * sde;
        acc[2] += J * sw;
        acc[3] += J * divw * sw;
        __builtin_amdgcn_wave_barrier();    // q, f reused by the wave's next element
    }
    for (int k = 0; k < kDiagSums; ++k) {
        const double s = block_sum(acc[k], s_red);
        if (threadIdx.x == 0) a.partial[int64_t(blockIdx.x) * kDiagSums + k] = s;
    }
}

// Final pass (one workgroup): sums of the partials in a fixed order, then
// out = {E_K, -dE_K/dt, |Omega|}.
__global__ void __launch_bounds__(kDiagBlock) energy_final_kernel(const double *partial, int nblocks, double rho_inf,
                                                                   double *out) {
    __shared__ double s_red[kDiagBlock];
    double tot[kDiagSums];
    for (int k = 0; k < kDiagSums; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[int64_t(b) * kDiagSums + k];
        tot[k] = block_sum(v, s_red);
    }
    if (threadIdx.x == 0) {
        const double vol = tot[2];
        const double ek = tot[0] / (rho_inf * vol);
        const double dek = (tot[1] - ek * rho_inf * tot[3]) / (rho_inf * vol);
        out[0] = ek;
        out[1] = -dek;
        out[2] = vol;
    }
}

// Wall force: one thread per wall face (list of element * Nfaces + face),
// one workgroup, fixed-order reduction.  out[0..DIM) pressure part,
// out[DIM..2 DIM) viscous part.
template <typename T>
struct ForceArgs {
    int nwall;
    const int32_t *wall;       // [nwall] element * Nfaces + face
    int Np, NF, Nfp;
    const T *Q;
    const int32_t *etov;
    const double *x;           // current vertex positions [nv][dim]
    const int32_t *fmask;      // [Nfaces][Nfp]
    const double *wface;       // [Nfaces][Nfp] integral of each face node's
                               // Lagrange function over a face of measure 2
    double c, rho0;
    double *out;
};

template <int DIM, typename T>
__global__ void __launch_bounds__(kDiagBlock) wall_force_kernel(ForceArgs<T> a) {
    __shared__ double s_red[kDiagBlock];
    double acc[2 * DIM];
    for (int k = 0; k < 2 * DIM; ++k) acc[k] = 0.0;
    const double c2 = a.c * a.c;
    for (int i = threadIdx.x; i < a.nwall; i += blockDim.x) {
        const int64_t e = a.wall[i] / (DIM + 1);
        const int f = a.wall[i] - int(e) * (DIM + 1);
        double xv[DIM + 1][DIM];
        for (int v = 0; v <= DIM; ++v) {
            const int64_t gv = a.etov[e * (DIM + 1) + v];
            for (int d = 0; d < DIM; ++d) xv[v][d] = a.x[gv * DIM + d];
        }
        // outward normal of the fluid element on face f and the face measure
        double n[DIM], meas;
        if constexpr (DIM == 2) {
            const int va = f, vb = (f + 1) % 3;
            const double tx = xv[vb][0] - xv[va][0], ty = xv[vb][1] - xv[va][1];
            meas = sqrt(tx * tx + ty * ty);
            n[0] = ty / meas;
            n[1] = -tx / meas;
        } else {
            const int fv[4][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {1, 2, 3, 0}, {0, 2, 3, 1}};
            const double *pa = xv[fv[f][0]], *pb = xv[fv[f][1]], *pc = xv[fv[f][2]], *po = xv[fv[f][3]];
            double u[3], v[3];
            for (int d = 0; d < 3; ++d) {
                u[d] = pb[d] - pa[d];
                v[d] = pc[d] - pa[d];
            }
            double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
            const double side = cr[0] * (pa[0] - po[0]) + cr[1] * (pa[1] - po[1]) + cr[2] * (pa[2] - po[2]);
            const double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            for (int d = 0; d < 3; ++d) n[d] = (side < 0.0 ? -cr[d] : cr[d]) / len;
            meas = 0.5 * len;
        }
        const double scale = 0.5 * meas;     // physical measure / reference measure 2
        for (int m = 0; m < a.Nfp; ++m) {
            const int j = a.fmask[f * a.Nfp + m];
            double qv[10];
            for (int k = 0; k < a.NF; ++k)
                qv[k] = double(a.Q[(((e >> 4) * a.NF + k) * a.Np + j) * 16 + (e & 15)]) + (k == 0 ? a.rho0 : 0.0);
            const double wgt = scale * a.wface[f * a.Nfp + m];
            const double rho = qv[0];
            double S[DIM][DIM];
            if constexpr (DIM == 2) {
                S[0][0] = kSqrt2 * qv[4];
                S[1][1] = kSqrt2 * qv[5];
                S[0][1] = S[1][0] = qv[3];
            } else {
                S[0][0] = kSqrt2 * qv[7];
                S[1][1] = kSqrt2 * qv[8];
                S[2][2] = kSqrt2 * qv[9];
                S[0][1] = S[1][0] = qv[4];
                S[0][2] = S[2][0] = qv[5];
                S[1][2] = S[2][1] = qv[6];
            }
            const double p = c2 * rho;
            for (int aa = 0; aa < DIM; ++aa) {
                double sn = 0.0;
                for (int b = 0; b < DIM; ++b) sn += -c2 * (S[aa][b] - qv[1 + aa] * qv[1 + b] / rho) * n[b];
                acc[aa] += wgt * p * n[aa];
                acc[DIM + aa] -= wgt * sn;
            }
        }
    }
    for (int k = 0; k < 2 * DIM; ++k) {
        const double s = block_sum(acc[k], s_red);
        if (threadIdx.x == 0) a.out[k] = s;
    }
}

// Equilibrium moments (Section 2) at every node: rho [K][Np], u [K][DIM][Np]
// (FP64) -> blocked state in T, density stored as rho - rho0; `offset`
// (NF values or null) is added to every node's moments.  Sets bit 0 of
// *bad for a non-positive density.
template <int DIM, typename T>
__global__ void equilibrium_kernel(const double *rho, const double *u, const double *offset, int64_t K, int Np,
                                   double c, double rho0, T *out, int *bad) {
    constexpr int NF = DIM == 2 ? 6 : 10;
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= K * Np) return;
    const int64_t e = idx / Np;
    const int j = int(idx - e * Np);
    const double r = rho[idx];
    if (!(r > 0.0)) {
        atomicOr(bad, 1);
        return;
    }
    double q[NF], m[DIM];
    for (int d = 0; d < DIM; ++d) m[d] = r * u[(e * DIM + d) * Np + j] / c;
    q[0] = r;
    for (int d = 0; d < DIM; ++d) q[1 + d] = m[d];
    if constexpr (DIM == 2) {
        q[3] = m[0] * m[1] / r;
        q[4] = m[0] * m[0] / (kSqrt2 * r);
        q[5] = m[1] * m[1] / (kSqrt2 * r);
    } else {
        q[4] = m[0] * m[1] / r;
        q[5] = m[0] * m[2] / r;
        q[6] = m[1] * m[2] / r;
        q[7] = m[0] * m[0] / (kSqrt2 * r);
        q[8] = m[1] * m[1] / (kSqrt2 * r);
        q[9] = m[2] * m[2] / (kSqrt2 * r);
    }
    for (int k = 0; k < NF; ++k) {
        const double v = q[k] + (offset ? offset[k] : 0.0) - (k == 0 ? rho0 : 0.0);
        out[(((e >> 4) * NF + k) * Np + j) * 16 + (e & 15)] = T(v);
    }
}

}  // namespace gbd
