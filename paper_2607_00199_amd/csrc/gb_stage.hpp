// Fused stage kernel of the ALE nodal DG Galerkin-Boltzmann method.
//
// One launch evaluates, for every element, the semi-discrete right-hand side
// F(q) of Section 3 (eq. semi_discrete_form, without the stiff -Lambda q part
// that Section 4 integrates exactly) at the geometry of one Runge-Kutta stage
// and stores that stage's SARK-4 combination:
//   geometry  vertex positions of the stage and the grid velocity (Section 5)
//             -> affine metrics, J, outward normals and sJ/J in FP64
//   volume    -c sum_d M_d d_d q + w . grad q  (eq. ale_bns)
//   surface   LIFT [ sJ/J  B~-(q- - q+) ]  (eq. upwind_flux)
//   source    P Ntilde(I q) on the stress fields (cubature)
//   update    the stage's SARK combination (four resident state arrays)
//
// Work decomposition: a workgroup holds EPB elements, Np threads each (one per
// node).  Reference operators are staged once per workgroup in LDS; each
// element's stage input is staged in LDS for the derivative, trace and
// cubature contractions.  Workgroups are persistent and take contiguous
// element ranges, with ranges assigned XCD by XCD so neighbour traces mostly
// hit the same L2.
//
// Upwinding: M_n (normal flux pattern) has spectrum in {-sqrt3,-1,0,1,sqrt3}
// for every unit normal (2D and the 3D tensor system), so the upwind matrix
// B~- = sum_lambda g(lambda) P_lambda is the degree-4 polynomial in M_n that
// interpolates g on those five points; g(lambda) = min(c lambda, 0) +
// min(-w.n, 0) (split) or min(c lambda - w.n, 0) (relative).
#pragma once

#include "gb_device.hpp"

namespace gbd {

enum StageKind { kStage0 = 0, kStage1 = 1, kStage2 = 2, kStage3 = 3, kRhsOnly = 4 };

template <typename T>
struct StageCoef {
    // decay factors exp(c_i gamma) and dt-scaled SARK weights of one field class
    T E1, E2, E3, E4;
    T a10, a20, a21, a30, a32;
    T b0, b1, b2, b3;
};

// Per-solver constants that change only with dt; kept in device memory and
// read through uniform loads.
template <typename T>
struct KConst {
    StageCoef<T> cf[2];  // [0] density/momentum (no relaxation), [1] stresses
    T c, inv_tau, rho0;
    int flux_mode;       // 0 split, 1 relative
    T fluxV[25];         // row p: coefficients of g -> power p of M_n
    T q_inf[10];
    int sponge;
    double sp_cx, sp_cy, sp_r0, sp_r1, sp_smax;
    double dt;
    Motion motion;
};

template <typename T>
struct KArgs {
    int64_t K;
    int nbatch;          // ceil(K / epb)
    int epb;             // elements per workgroup
    int Nc;              // cubature points
    int chunk;           // batches per workgroup
    const int32_t *etov;
    const double *xs;    // vertex positions of this stage [nv][DIM]
    const double *ws;    // grid velocity at the vertices for this stage [nv][DIM]
    const int32_t *vmapP;
    const T *ops;        // packed reference operators (see OpOffsets)
    const int32_t *fmask;
    T *Q, *A, *B, *G;    // state arrays of the SARK-4 schedule
    const double *clock; // [0] = t_n
    const KConst<T> *kc;
    int *err;            // bit 0: J <= 0, bit 1: density <= 0 or NaN
};

template <int DIM, int N>
struct Shape {
    static constexpr int NP = DIM == 2 ? (N + 1) * (N + 2) / 2 : (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int NFACES = DIM + 1;
    static constexpr int NFP = DIM == 2 ? N + 1 : (N + 1) * (N + 2) / 2;
    static constexpr int NFT = NFACES * NFP;
    static constexpr int NF = DIM == 2 ? 6 : 10;
    static constexpr int NCONS = DIM + 1;
    static constexpr int NS = NF - NCONS;
    static constexpr int NVERT = DIM + 1;
    static constexpr int GEO = DIM * DIM + NFACES * DIM + NFACES + 2 * NVERT * DIM;
    // offsets inside GEO
    static constexpr int G_MET = 0;
    static constexpr int G_NRM = DIM * DIM;
    static constexpr int G_FSC = G_NRM + NFACES * DIM;
    static constexpr int G_WV = G_FSC + NFACES;
    static constexpr int G_XV = G_WV + NVERT * DIM;
};

// Packed operator layout (all of type T):
//   DT    [DIM][NP][NP]   DT[a][j][i] = D_a(i, j)
//   LIFTT [NFT][NP]       LIFTT[m][i] = LIFT(i, m)
//   IcT   [NP][Nc]        IcT[j][k]  = Icub(k, j)
//   PcT   [Nc][NP]        PcT[k][i]  = Pcub(i, k)
//   BARY  [NP][NVERT]
template <int DIM, int N>
struct OpOffsets {
    using S = Shape<DIM, N>;
    __host__ __device__ static constexpr int dt() { return 0; }
    __host__ __device__ static constexpr int lift() { return DIM * S::NP * S::NP; }
    __host__ __device__ static constexpr int ic() { return lift() + S::NFT * S::NP; }
    __host__ __device__ static int pc(int Nc) { return ic() + S::NP * Nc; }
    __host__ __device__ static int bary(int Nc) { return pc(Nc) + Nc * S::NP; }
    __host__ __device__ static int total(int Nc) { return bary(Nc) + S::NP * S::NVERT; }
};

template <int DIM, int N>
__host__ __device__ inline int sbuf_size(int Nc) {
    using S = Shape<DIM, N>;
    const int a = S::NF * S::NFT, b = S::NS * Nc;
    return a > b ? a : b;
}

// LDS bytes for a workgroup of `epb` elements.
template <int DIM, int N, typename T>
inline size_t lds_bytes(int Nc, int epb) {
    using S = Shape<DIM, N>;
    size_t ops = size_t(OpOffsets<DIM, N>::total(Nc)) * sizeof(T);
    ops = (ops + 15) / 16 * 16;
    size_t fm = size_t(S::NFT) * sizeof(int32_t);
    fm = (fm + 15) / 16 * 16;
    const size_t per = size_t(S::NF * S::NP + sbuf_size<DIM, N>(Nc) + S::GEO) * sizeof(T);
    return ops + fm + per * epb;
}

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

// Stage input at flat node index (e*NP + j), field k, formed from the
// resident arrays for the stage being evaluated.
template <int DIM, int N, int STAGE, typename T>
__device__ __forceinline__ T stage_input(const KArgs<T> &a, int64_t base, int k) {
    using S = Shape<DIM, N>;
    const int64_t addr = base + int64_t(k) * S::NP;
    if constexpr (STAGE == kStage0 || STAGE == kRhsOnly) {
        return a.Q[addr];
    } else if constexpr (STAGE == kStage1) {
        const StageCoef<T> &c = a.kc->cf[k < S::NCONS ? 0 : 1];
        return c.E1 * a.Q[addr] + c.a10 * a.A[addr];
    } else if constexpr (STAGE == kStage2) {
        return a.B[addr];
    } else {
        return a.A[addr];
    }
}

template <int DIM, int N, typename T, int STAGE>
__global__ void __launch_bounds__(256) stage_kernel(KArgs<T> a) {
    using S = Shape<DIM, N>;
    using O = OpOffsets<DIM, N>;
    constexpr int NP = S::NP, NF = S::NF, NFT = S::NFT, NFP = S::NFP, NCONS = S::NCONS, NS = S::NS;
    constexpr int NVERT = S::NVERT, GEO = S::GEO;
    const int Nc = a.Nc;
    const int SB = sbuf_size<DIM, N>(Nc);

    extern __shared__ __align__(16) unsigned char smem[];
    T *s_ops = reinterpret_cast<T *>(smem);
    size_t off = (size_t(O::total(Nc)) * sizeof(T) + 15) / 16 * 16;
    int32_t *s_fmask = reinterpret_cast<int32_t *>(smem + off);
    off += (size_t(NFT) * sizeof(int32_t) + 15) / 16 * 16;
    T *s_q = reinterpret_cast<T *>(smem + off);               // [epb][NF][NP]
    T *s_buf = s_q + size_t(a.epb) * NF * NP;                  // [epb][SB]
    T *s_geo = s_buf + size_t(a.epb) * SB;                     // [epb][GEO]

    const T *DT = s_ops + O::dt();
    const T *LIFTT = s_ops + O::lift();
    const T *IcT = s_ops + O::ic();
    const T *PcT = s_ops + O::pc(Nc);
    const T *BARY = s_ops + O::bary(Nc);

    const int tid = threadIdx.x;
    for (int p = tid; p < O::total(Nc); p += blockDim.x) s_ops[p] = a.ops[p];
    for (int p = tid; p < NFT; p += blockDim.x) s_fmask[p] = a.fmask[p];

    const int el = tid / NP;
    const int i = tid - el * NP;
    const bool lane_ok = el < a.epb;

    // contiguous batch range per workgroup, ranges laid out XCD by XCD
    int logical = blockIdx.x;
    if ((gridDim.x & 7) == 0) logical = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int b_begin = logical * a.chunk;
    int b_end = b_begin + a.chunk;
    if (b_end > a.nbatch) b_end = a.nbatch;

    const KConst<T> &kc = *a.kc;
    // partial unrolling keeps the contraction loops from hoisting every LDS
    // load into registers
    constexpr int UNR = sizeof(T) == 8 ? 2 : 4;
    __syncthreads();

    for (int batch = b_begin; batch < b_end; ++batch) {
        const int64_t e = int64_t(batch) * a.epb + el;
        const bool active = lane_ok && e < a.K;
        T *q_el = s_q + size_t(el) * NF * NP;
        T *buf_el = s_buf + size_t(el) * SB;
        T *geo = s_geo + size_t(el) * GEO;

        // ---- geometry of the stage, FP64, one thread per element
        if (active && i == 0) {
            double xv[NVERT][DIM], wv[NVERT][DIM];
            for (int v = 0; v < NVERT; ++v) {
                const int64_t gv = a.etov[e * NVERT + v];
                for (int d = 0; d < DIM; ++d) {
                    xv[v][d] = a.xs[gv * DIM + d];
                    wv[v][d] = a.ws[gv * DIM + d];
                }
            }
            double Gm[DIM][DIM];  // Gm[i][a] = dx_i/dr_a
            for (int ii = 0; ii < DIM; ++ii)
                for (int aa = 0; aa < DIM; ++aa) Gm[ii][aa] = 0.5 * (xv[aa + 1][ii] - xv[0][ii]);
            double J, inv[DIM][DIM];  // inv[a][i] = dr_a/dx_i
            if constexpr (DIM == 2) {
                J = Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0];
                inv[0][0] = Gm[1][1] / J;
                inv[0][1] = -Gm[0][1] / J;
                inv[1][0] = -Gm[1][0] / J;
                inv[1][1] = Gm[0][0] / J;
            } else {
                const double c00 = Gm[1][1] * Gm[2][2] - Gm[1][2] * Gm[2][1];
                const double c01 = Gm[1][2] * Gm[2][0] - Gm[1][0] * Gm[2][2];
                const double c02 = Gm[1][0] * Gm[2][1] - Gm[1][1] * Gm[2][0];
                J = Gm[0][0] * c00 + Gm[0][1] * c01 + Gm[0][2] * c02;
                inv[0][0] = c00 / J;
                inv[1][0] = c01 / J;
                inv[2][0] = c02 / J;
                inv[0][1] = (Gm[0][2] * Gm[2][1] - Gm[0][1] * Gm[2][2]) / J;
                inv[1][1] = (Gm[0][0] * Gm[2][2] - Gm[0][2] * Gm[2][0]) / J;
                inv[2][1] = (Gm[0][1] * Gm[2][0] - Gm[0][0] * Gm[2][1]) / J;
                inv[0][2] = (Gm[0][1] * Gm[1][2] - Gm[0][2] * Gm[1][1]) / J;
                inv[1][2] = (Gm[0][2] * Gm[1][0] - Gm[0][0] * Gm[1][2]) / J;
                inv[2][2] = (Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0]) / J;
            }
            if (!(J > 0.0)) atomicOr(a.err, 1);
            for (int aa = 0; aa < DIM; ++aa)
                for (int ii = 0; ii < DIM; ++ii) geo[S::G_MET + aa * DIM + ii] = T(inv[aa][ii]);
            if constexpr (DIM == 2) {
                for (int f = 0; f < 3; ++f) {
                    const int va = f, vb = (f + 1) % 3;
                    const double tx = xv[vb][0] - xv[va][0], ty = xv[vb][1] - xv[va][1];
                    const double len = sqrt(tx * tx + ty * ty);
                    geo[S::G_NRM + 2 * f] = T(ty / len);
                    geo[S::G_NRM + 2 * f + 1] = T(-tx / len);
                    geo[S::G_FSC + f] = T(0.5 * len / J);
                }
            } else {
                const int fv[4][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {1, 2, 3, 0}, {0, 2, 3, 1}};
                for (int f = 0; f < 4; ++f) {
                    const double *pa = xv[fv[f][0]], *pb = xv[fv[f][1]], *pc = xv[fv[f][2]], *po = xv[fv[f][3]];
                    const double u0 = pb[0] - pa[0], u1 = pb[1] - pa[1], u2 = pb[2] - pa[2];
                    const double v0 = pc[0] - pa[0], v1 = pc[1] - pa[1], v2 = pc[2] - pa[2];
                    double n0 = u1 * v2 - u2 * v1, n1 = u2 * v0 - u0 * v2, n2 = u0 * v1 - u1 * v0;
                    if (n0 * (pa[0] - po[0]) + n1 * (pa[1] - po[1]) + n2 * (pa[2] - po[2]) < 0.0) {
                        n0 = -n0;
                        n1 = -n1;
                        n2 = -n2;
                    }
                    const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
                    geo[S::G_NRM + 3 * f] = T(n0 / nn);
                    geo[S::G_NRM + 3 * f + 1] = T(n1 / nn);
                    geo[S::G_NRM + 3 * f + 2] = T(n2 / nn);
                    geo[S::G_FSC + f] = T(0.25 * nn / J);   // sJ = area / 2 = |n| / 4
                }
            }
            for (int v = 0; v < NVERT; ++v)
                for (int d = 0; d < DIM; ++d) {
                    geo[S::G_WV + v * DIM + d] = T(wv[v][d]);
                    geo[S::G_XV + v * DIM + d] = T(xv[v][d]);
                }
        }

        // ---- stage input of this thread's node into LDS
        const int64_t base = active ? (e * NF * NP + i) : 0;
        if (active) {
#pragma unroll
            for (int k = 0; k < NF; ++k) q_el[k * NP + i] = stage_input<DIM, N, STAGE, T>(a, base, k);
        }
        __syncthreads();

        T rhs[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) rhs[k] = T(0);
        if (active) {
            // ---- volume term: reference derivatives, chain rule, -c M_d + w_d
            T dr[DIM][NF];
#pragma unroll
            for (int aa = 0; aa < DIM; ++aa)
#pragma unroll
                for (int k = 0; k < NF; ++k) dr[aa][k] = T(0);
#pragma unroll UNR
            for (int j = 0; j < NP; ++j) {
                T dcoef[DIM];
#pragma unroll
                for (int aa = 0; aa < DIM; ++aa) dcoef[aa] = DT[(aa * NP + j) * NP + i];
#pragma unroll
                for (int k = 0; k < NF; ++k) {
                    const T qv = q_el[k * NP + j];
#pragma unroll
                    for (int aa = 0; aa < DIM; ++aa) dr[aa][k] += dcoef[aa] * qv;
                }
            }
#pragma unroll
            for (int ii = 0; ii < DIM; ++ii) {
                T wnode = T(0);
#pragma unroll
                for (int v = 0; v < NVERT; ++v) wnode += BARY[i * NVERT + v] * geo[S::G_WV + v * DIM + ii];
                T g[NF];
#pragma unroll
                for (int k = 0; k < NF; ++k) {
                    T sum = T(0);
#pragma unroll
                    for (int aa = 0; aa < DIM; ++aa) sum += geo[S::G_MET + aa * DIM + ii] * dr[aa][k];
                    g[k] = sum;
                    rhs[k] += wnode * sum;
                }
                if (ii == 0) sub_cMd<DIM, 0, T>(kc.c, g, rhs);
                if (ii == 1) sub_cMd<DIM, 1, T>(kc.c, g, rhs);
                if constexpr (DIM == 3)
                    if (ii == 2) sub_cMd<DIM, 2, T>(kc.c, g, rhs);
            }

            // ---- surface fluxes at the face nodes
#pragma unroll 1
            for (int m = i; m < NFT; m += NP) {
                const int f = m / NFP;
                const int vm = s_fmask[m];
                const int32_t idx = a.vmapP[e * NFT + m];
                T y[NF];
                if (idx >= 0) {
                    const int64_t nb = int64_t(idx);
                    const int64_t ne = nb / NP;
                    const int64_t nbase = ne * NF * NP + (nb - ne * NP);
#pragma unroll
                    for (int k = 0; k < NF; ++k) y[k] = q_el[k * NP + vm] - stage_input<DIM, N, STAGE, T>(a, nbase, k);
                } else if (idx == -1) {
                    // moving no-slip wall: ghost density and stresses mirror the
                    // interior, momentum is reflected about the wall velocity
#pragma unroll
                    for (int k = 0; k < NF; ++k) y[k] = T(0);
#pragma unroll
                    for (int d = 0; d < DIM; ++d) {
                        T wd = T(0);
#pragma unroll
                        for (int v = 0; v < NVERT; ++v) wd += BARY[vm * NVERT + v] * geo[S::G_WV + v * DIM + d];
                        const T mm = q_el[(1 + d) * NP + vm];
                        y[1 + d] = mm - (T(2) * (q_el[vm] + kc.rho0) * wd / kc.c - mm);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NF; ++k) y[k] = q_el[k * NP + vm] - kc.q_inf[k];
                }
                T nrm[DIM], wn = T(0);
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    nrm[d] = geo[S::G_NRM + f * DIM + d];
                    T wd = T(0);
#pragma unroll
                    for (int v = 0; v < NVERT; ++v) wd += BARY[vm * NVERT + v] * geo[S::G_WV + v * DIM + d];
                    wn += wd * nrm[d];
                }
                // weights g(lambda) on the spectrum {-sqrt3, -1, 0, 1, sqrt3}
                T gl[5];
                {
                    const T cs3 = kc.c * T(1.7320508075688772);
                    const T lam[5] = {-cs3, -kc.c, T(0), kc.c, cs3};
                    const T wneg = tmin(-wn, T(0));
#pragma unroll
                    for (int l = 0; l < 5; ++l)
                        gl[l] = kc.flux_mode == 0 ? tmin(lam[l], T(0)) + wneg : tmin(lam[l] - wn, T(0));
                }
                T acc[NF];
                T cp = T(0);
#pragma unroll
                for (int l = 0; l < 5; ++l) cp += kc.fluxV[l] * gl[l];
#pragma unroll
                for (int k = 0; k < NF; ++k) acc[k] = cp * y[k];
#pragma unroll
                for (int p = 1; p < 5; ++p) {
                    T z[NF];
                    apply_Mn<DIM, T>(nrm, y, z);
                    cp = T(0);
#pragma unroll
                    for (int l = 0; l < 5; ++l) cp += kc.fluxV[p * 5 + l] * gl[l];
#pragma unroll
                    for (int k = 0; k < NF; ++k) {
                        y[k] = z[k];
                        acc[k] += cp * z[k];
                    }
                }
                const T fs = geo[S::G_FSC + f];
#pragma unroll
                for (int k = 0; k < NF; ++k) buf_el[k * NFT + m] = fs * acc[k];
            }
        }
        __syncthreads();
        if (active) {
            // ---- lift
#pragma unroll UNR
            for (int m = 0; m < NFT; ++m) {
                const T l = LIFTT[m * NP + i];
#pragma unroll
                for (int k = 0; k < NF; ++k) rhs[k] += l * buf_el[k * NFT + m];
            }
        }
        __syncthreads();
        if (active) {
            // ---- relaxation source at the cubature points
#pragma unroll 1
            for (int kq = i; kq < Nc; kq += NP) {
                T qc[NCONS];
#pragma unroll
                for (int c = 0; c < NCONS; ++c) qc[c] = T(0);
#pragma unroll UNR
                for (int j = 0; j < NP; ++j) {
                    const T w = IcT[j * Nc + kq];
#pragma unroll
                    for (int c = 0; c < NCONS; ++c) qc[c] += w * q_el[c * NP + j];
                }
                T nt[NS];
                ntilde<DIM, T>(qc[0] + kc.rho0, qc + 1, kc.inv_tau, nt);
#pragma unroll
                for (int s = 0; s < NS; ++s) buf_el[s * Nc + kq] = nt[s];
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll UNR
            for (int kq = 0; kq < Nc; ++kq) {
                const T p = PcT[kq * NP + i];
#pragma unroll
                for (int s = 0; s < NS; ++s) rhs[NCONS + s] += p * buf_el[s * Nc + kq];
            }
            // ---- sponge layer (absorbing-layer stand-in)
            if constexpr (DIM == 2) {
                if (kc.sponge) {
                    double px = 0.0, py = 0.0;
                    for (int v = 0; v < NVERT; ++v) {
                        px += double(BARY[i * NVERT + v]) * double(geo[S::G_XV + v * DIM + 0]);
                        py += double(BARY[i * NVERT + v]) * double(geo[S::G_XV + v * DIM + 1]);
                    }
                    const double r = sqrt((px - kc.sp_cx) * (px - kc.sp_cx) + (py - kc.sp_cy) * (py - kc.sp_cy));
                    double xi = (r - kc.sp_r0) / (kc.sp_r1 - kc.sp_r0);
                    xi = xi < 0.0 ? 0.0 : (xi > 1.0 ? 1.0 : xi);
                    const T sig = T(kc.sp_smax * xi * xi);
#pragma unroll
                    for (int k = 0; k < NF; ++k) rhs[k] -= sig * (q_el[k * NP + i] - kc.q_inf[k]);
                }
            }

            // ---- SARK-4 stage combination and store
#pragma unroll
            for (int k = 0; k < NF; ++k) {
                const StageCoef<T> &c = kc.cf[k < NCONS ? 0 : 1];
                const int64_t addr = base + int64_t(k) * NP;
                if constexpr (STAGE == kRhsOnly || STAGE == kStage0) {
                    a.A[addr] = rhs[k];
                } else if constexpr (STAGE == kStage1) {
                    const T qn = a.Q[addr], f0 = a.A[addr];
                    a.B[addr] = c.E2 * qn + c.a20 * f0 + c.a21 * rhs[k];
                    a.G[addr] = c.E4 * qn + c.b0 * f0 + c.b1 * rhs[k];
                } else if constexpr (STAGE == kStage2) {
                    const T qn = a.Q[addr], f0 = a.A[addr], g = a.G[addr];
                    a.A[addr] = c.E3 * qn + c.a30 * f0 + c.a32 * rhs[k];
                    a.G[addr] = g + c.b2 * rhs[k];
                } else {
                    const T v = a.G[addr] + c.b3 * rhs[k];
                    a.Q[addr] = v;
                    if (k == 0) {
                        const T rho = v + kc.rho0;
                        if (!(rho > T(0))) atomicOr(a.err, 2);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Vertex data of the four Runge-Kutta stages of one step (Section 5: vertex
// coordinates advance with the classical RK4 scheme on dx/dt = v_G(X, t), and
// the grid velocity is prescribed at the vertices).  The right-hand side of
// that ODE depends on (X, t) only, so the RK4 slopes are the velocities at the
// stage times:
//   x_n0 = x_n,  x_n1 = x_n + dt/2 w(t_n),  x_n2 = x_n + dt/2 w(t_n + dt/2),
//   x_n3 = x_n + dt w(t_n + dt/2),
//   x_{n+1} = x_n + dt (w(t_n) + 2 w(t_n+dt/2) + 2 w(t_n+dt/2) + w(t_n+dt)) / 6
// and stage j uses the velocity w(t_n + c_j dt), c = (0, 1/2, 1/2, 1).
// Writes xs[s][nv][DIM] for s = 0..4 (4 = end of step) and ws[s][nv][DIM]
// for s = 0..3.
template <int DIM>
__global__ void motion_stages_kernel(int64_t nv, const double *X, const double *x, const double *clock, double dt,
                                     Motion m, double *xs, double *ws) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const double tn = clock[0];
    double Xv[DIM], xn[DIM], w0[DIM], w1[DIM], w2[DIM], w3[DIM];
    for (int d = 0; d < DIM; ++d) {
        Xv[d] = X[v * DIM + d];
        xn[d] = x[v * DIM + d];
    }
    motion_velocity<DIM>(m, Xv, tn, w0);
    motion_velocity<DIM>(m, Xv, tn + 0.5 * dt, w1);
    motion_velocity<DIM>(m, Xv, tn + 0.5 * dt, w2);
    motion_velocity<DIM>(m, Xv, tn + 1.0 * dt, w3);
    const int64_t st = nv * DIM;
    for (int d = 0; d < DIM; ++d) {
        const int64_t o = v * DIM + d;
        xs[0 * st + o] = xn[d];
        xs[1 * st + o] = xn[d] + 0.5 * dt * w0[d];
        xs[2 * st + o] = xn[d] + 0.5 * dt * w1[d];
        xs[3 * st + o] = xn[d] + dt * w2[d];
        xs[4 * st + o] = xn[d] + dt * (w0[d] + 2.0 * w1[d] + 2.0 * w2[d] + w3[d]) / 6.0;
        ws[0 * st + o] = w0[d];
        ws[1 * st + o] = w1[d];
        ws[2 * st + o] = w2[d];
        ws[3 * st + o] = w3[d];
    }
}

// End of a step: x_n <- x_{n+1}; the first thread also advances the clock.
template <int DIM>
__global__ void finish_step_kernel(int64_t nv, double *x, const double *xnext, double *clock, double dt) {
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v < nv)
        for (int d = 0; d < DIM; ++d) x[v * DIM + d] = xnext[v * DIM + d];
    if (v == 0) {
        clock[0] = clock[0] + dt;
        clock[1] = clock[1] + 1.0;
    }
}

}  // namespace gbd
