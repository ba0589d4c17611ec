// Fused stage kernel, matrix-core form.
//
// Same arithmetic as the per-stage right-hand side and SARK-4 update of
// Sections 3-5 of the paper (see gb_stage.hpp for the term list), organised
// for the CDNA4 matrix cores:
//
//   * one wavefront owns 16 elements; they are the 16 columns of every
//     16x16x4 MFMA (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64), so all
//     four contractions of a stage are matrix products with the element index
//     as the N dimension:
//       volume      dq/dr_a [node, elem]    = D_a  [node, node]     q [node, elem]
//       lift        rhs     [node, elem]   += LIFT [node, facenode] flux[facenode, elem]
//       cubature    q_c     [point, elem]   = I    [point, node]    q [node, elem]
//       projection  rhs     [node, elem]   += P    [node, point]    Nt[point, elem]
//   * operator fragments (the A operands, one value per lane per MFMA) are
//     staged once per workgroup in LDS in lane order; the B operands are read
//     straight from HBM (state in the blocked layout [K/16][NF][Np][16], so a
//     fragment load is 16 consecutive elements per node row) or computed in
//     registers (face fluxes, Ntilde at the cubature points), always in the
//     lane that the MFMA consumes them from, so no data moves between lanes;
//   * the accumulator fragment of a lane holds four node rows of one element;
//     the point-wise work (chain rule, flux mixing, ALE term, SARK combination)
//     is done there, in registers.
// The contraction index of the projection is ordered to match the
// accumulator layout of the cubature product, so Ntilde never changes lanes.
#pragma once

#include "gb_stage.hpp"

namespace gbd {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    using type = f4v;
};
template <>
struct Vec4<double> {
    using type = d4v;
};

__device__ __forceinline__ f4v mfma16(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16x16 accumulator held in slot r by the lanes with lane/16 == q
// (measured lane layout on gfx950: FP32 rows 4q + r, FP64 rows q + 4r).
template <typename T>
__host__ __device__ constexpr int crow(int q, int r) {
    return sizeof(T) == 4 ? 4 * q + r : q + 4 * r;
}

// Entry (row, col) of the flux pattern M_d (A_d = -c M_d).
template <int DIM>
__host__ __device__ constexpr double mcoef(int d, int row, int col) {
    constexpr double s2 = 1.41421356237309504880;
    if (DIM == 2) {
        if (d == 0) {
            if ((row == 0 && col == 1) || (row == 1 && col == 0) || (row == 2 && col == 3) || (row == 3 && col == 2))
                return 1.0;
            if ((row == 1 && col == 4) || (row == 4 && col == 1)) return s2;
            return 0.0;
        }
        if ((row == 0 && col == 2) || (row == 1 && col == 3) || (row == 2 && col == 0) || (row == 3 && col == 1))
            return 1.0;
        if ((row == 2 && col == 5) || (row == 5 && col == 2)) return s2;
        return 0.0;
    }
    // 3D: rho 0, m 1..3, Sxy 4, Sxz 5, Syz 6, S_ii/sqrt2 7..9
    const int m = 1 + d;
    if ((row == 0 && col == m) || (row == m && col == 0)) return 1.0;
    if ((row == m && col == 7 + d) || (row == 7 + d && col == m)) return s2;
    // off-diagonal stresses: S_ij couples to m_i through d_j and to m_j through d_i
    const int off[3][3] = {{-1, 4, 5}, {4, -1, 6}, {5, 6, -1}};
    for (int i = 0; i < 3; ++i) {
        if (i == d) continue;
        const int sidx = off[i][d];
        if ((row == 1 + i && col == sidx) || (row == sidx && col == 1 + i)) return 1.0;
    }
    return 0.0;
}

template <int DIM, int N>
struct MShape {
    using S = Shape<DIM, N>;
    static constexpr int NJS = (S::NP + 3) / 4;    // k-steps over nodes
    static constexpr int NRT = (S::NP + 15) / 16;  // 16-row tiles over nodes
    static constexpr int NMS = (S::NFT + 3) / 4;   // k-steps over face nodes
};

// Packed operator fragments (type T, 64 lane-ordered values per fragment):
//   FD [DIM][NRT][NJS]   lane (q, c): D_a(16 rt + c, 4 s + q)
//   FL [NRT][NMS]        LIFT(16 rt + c, 4 s + q)
//   FI [NCT][NJS]        Icub(16 t + c, 4 s + q)
//   FP [NRT][NCT][4]     Pcub(16 rt + c, 16 t + crow(q, r))
//   BARY [NP][NVERT]
// then an int table SLOT [4 NMS][2]: (volume node, face) of face slot m, or -1.
template <int DIM, int N>
struct MOps {
    using M = MShape<DIM, N>;
    using S = Shape<DIM, N>;
    __host__ __device__ static constexpr int fd(int a, int rt, int s) { return ((a * M::NRT + rt) * M::NJS + s) * 64; }
    __host__ __device__ static constexpr int fl(int rt, int s) { return (DIM * M::NRT * M::NJS + rt * M::NMS + s) * 64; }
    __host__ __device__ static constexpr int fi_base() { return (DIM * M::NRT * M::NJS + M::NRT * M::NMS) * 64; }
    __host__ __device__ static int fi(int nct, int t, int s) { (void)nct; return fi_base() + (t * M::NJS + s) * 64; }
    __host__ __device__ static int fp(int nct, int rt, int t, int r) {
        return fi_base() + nct * M::NJS * 64 + ((rt * nct + t) * 4 + r) * 64;
    }
    __host__ __device__ static int bary(int nct) { return fi_base() + nct * M::NJS * 64 + M::NRT * nct * 4 * 64; }
    __host__ __device__ static int total(int nct) { return bary(nct) + S::NP * S::NVERT; }
    __host__ __device__ static constexpr int slots() { return 4 * M::NMS; }
};

// Workgroup LDS: operator fragments, the slot table, then one stage-input
// block [NF][Np][16] per wavefront (kWaves wavefronts of 64 lanes).
constexpr int kWaves = 4;

template <int DIM, int N, typename T>
__host__ __device__ inline size_t mfma_lds_state_offset(int nct) {
    size_t b = size_t(MOps<DIM, N>::total(nct)) * sizeof(T);
    b = (b + 15) / 16 * 16;
    b += size_t(MOps<DIM, N>::slots()) * 2 * sizeof(int32_t);
    return (b + 15) / 16 * 16;
}

// The stage-input block is staged in LDS unless the operators already take
// most of it (tetrahedra of order 3 in FP64: about 80 KB of fragments).
template <int DIM, int N, typename T>
__host__ __device__ constexpr bool stage_in_lds() {
    return !(DIM == 3 && N >= 3 && sizeof(T) == 8);
}

template <int DIM, int N, typename T>
inline size_t mfma_lds_bytes(int nct) {
    using S = Shape<DIM, N>;
    const size_t state = stage_in_lds<DIM, N, T>() ? size_t(kWaves) * S::NF * S::NP * 16 * sizeof(T) : 0;
    return mfma_lds_state_offset<DIM, N, T>(nct) + state;
}

// Blocked state address of (element e, field k, node j).
template <int NF, int NP>
__device__ __forceinline__ int64_t baddr(int64_t e, int k, int j) {
    return ((((e >> 4) * NF + k) * NP + j) << 4) + (e & 15);
}

// Stage input of field k at a blocked offset `off` (relative to the state
// arrays' common base), formed from the resident arrays for the stage being
// evaluated.
template <int NCONS, int STAGE, typename T>
__device__ __forceinline__ T stage_in_at(const T *Q, const T *A, const T *B, const KConst<T> &kc, int k, int64_t off) {
    if constexpr (STAGE == kStage0 || STAGE == kRhsOnly) {
        return Q[off];
    } else if constexpr (STAGE == kStage1) {
        const StageCoef<T> &c = kc.cf[k < NCONS ? 0 : 1];
        return c.E1 * Q[off] + c.a10 * A[off];
    } else if constexpr (STAGE == kStage2) {
        (void)Q;
        return B[off];
    } else {
        return A[off];
    }
}

// Occupancy target: two wavefronts per SIMD for the FP32 triangle kernels
// with one 16-row node tile (their registers fit that budget without
// spills); the others need the whole register file.
template <int DIM, int N>
__host__ __device__ constexpr int stage_waves_per_eu(int elem_bytes) {
    return (elem_bytes == 4 && DIM == 2 && MShape<DIM, N>::NRT == 1) ? 2 : 1;
}

template <int DIM, int N, typename T, int STAGE>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<DIM, N>(sizeof(T)))))
stage_mfma_kernel(KArgs<T> a) {
    using S = Shape<DIM, N>;
    using MS = MShape<DIM, N>;
    using O = MOps<DIM, N>;
    using V = typename Vec4<T>::type;
    constexpr int NP = S::NP, NF = S::NF, NFT = S::NFT, NCONS = S::NCONS, NS = S::NS, NVERT = S::NVERT;
    constexpr int NFACES = S::NFACES, NJS = MS::NJS, NRT = MS::NRT, NMS = MS::NMS;
    const int Nc = a.Nc;
    const int nct = (Nc + 15) / 16;

    extern __shared__ __align__(16) unsigned char smem[];
    T *s_ops = reinterpret_cast<T *>(smem);
    const int nops = O::total(nct);
    int32_t *s_slot = reinterpret_cast<int32_t *>(smem + (size_t(nops) * sizeof(T) + 15) / 16 * 16);
    for (int p = threadIdx.x; p < nops; p += blockDim.x) s_ops[p] = a.ops[p];
    for (int p = threadIdx.x; p < 2 * O::slots(); p += blockDim.x) s_slot[p] = a.fmask[p];
    __syncthreads();

    const KConst<T> &kc = *a.kc;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
    const int col = lane & 15;
    const int q4 = lane >> 4;
    const T *BARY = s_ops + O::bary(nct);
    constexpr int BLK = NF * NP * 16;
    T *s_q = reinterpret_cast<T *>(smem + mfma_lds_state_offset<DIM, N, T>(nct)) + wave * BLK;

    int logical = blockIdx.x;
    if ((gridDim.x & 7) == 0) logical = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int g_begin = logical * a.chunk;
    int g_end = g_begin + a.chunk;
    if (g_end > a.nbatch) g_end = a.nbatch;

    for (int gi = g_begin + wave; gi < g_end; gi += nwave) {
        const int g = __builtin_amdgcn_readfirstlane(gi);
        const int64_t e = int64_t(g) * 16 + col;
        const bool valid = e < a.K;
        // wave-uniform bases of this group's block in the state arrays; lanes
        // address them with 32-bit offsets (k NP + j) 16 + col
        constexpr int GSTRIDE = NF * NP * 16;
        const int64_t gbase = int64_t(g) * GSTRIDE;
        const T *Qg = a.Q + gbase, *Ag = a.A + gbase, *Bg = a.B + gbase;
        T *Qw = a.Q + gbase, *Aw = a.A + gbase, *Bw = a.B + gbase, *Gw = a.G + gbase;

        // ---- loads, issued together so that a group costs the wave about
        //      three memory round trips rather than one per operand: trace
        //      map and vertex ids; the group's stage input (one contiguous
        //      block) copied to this wave's LDS; the first face slot's
        //      neighbour values and the stage vertex data
        const int32_t *vmg = a.vmapP + int64_t(g) * (O::slots() * 16) + q4 * 16 + col;
        int32_t vm_cur = vmg[0];
        int32_t vm_nxt = NMS > 1 ? vmg[64] : 0;
        int32_t vid[NVERT];
#pragma unroll
        for (int v = 0; v < NVERT; ++v) vid[v] = valid ? a.etov[e * NVERT + v] : 0;
        constexpr bool LDS_IN = stage_in_lds<DIM, N, T>();
        if constexpr (LDS_IN) {
#pragma unroll
            for (int k = 0; k < NF; ++k)
#pragma unroll
                for (int p = lane; p < NP * 16; p += 64)
                    s_q[k * NP * 16 + p] = stage_in_at<NCONS, STAGE, T>(Qg, Ag, Bg, kc, k, k * NP * 16 + p);
        }
        // neighbour values of face slot s2 (boundary and padding slots read
        // this lane's own, always allocated, node: every load is in bounds)
        auto gather = [&](int s2, int32_t idx, T *out) {
            const int vm = s_slot[2 * (4 * s2 + q4)];
            int64_t off = gbase + (vm > 0 ? vm : 0) * 16 + col;
            if (idx >= 0) {
                const int e2 = idx / NP;
                const int j2 = idx - e2 * NP;
                off = (int64_t(e2 >> 4) * (NF * NP) + j2) * 16 + (e2 & 15);
            }
#pragma unroll
            for (int k = 0; k < NF; ++k) out[k] = stage_in_at<NCONS, STAGE, T>(a.Q, a.A, a.B, kc, k, off + k * NP * 16);
        };
        T nb_cur[NF];
        gather(0, vm_cur, nb_cur);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        auto own = [&](int k, int j) -> T {
            if constexpr (LDS_IN)
                return s_q[(k * NP + j) * 16 + col];
            else
                return stage_in_at<NCONS, STAGE, T>(Qg, Ag, Bg, kc, k, (k * NP + j) * 16 + col);
        };

        // ---- geometry of this lane's element (FP64; the four lanes of an
        //      element compute it redundantly)
        T met[DIM * DIM], nrm[NFACES * DIM], fsc[NFACES], wvt[NVERT * DIM];
        {
            double xv[NVERT][DIM], wv[NVERT][DIM];
            for (int v = 0; v < NVERT; ++v) {
                const int64_t gv = vid[v];
                for (int d = 0; d < DIM; ++d) {
                    xv[v][d] = valid ? a.xs[gv * DIM + d] : (v == d + 1 ? 1.0 : 0.0);
                    wv[v][d] = valid ? a.ws[gv * DIM + d] : 0.0;
                }
            }
            double Gm[DIM][DIM];
            for (int ii = 0; ii < DIM; ++ii)
                for (int aa = 0; aa < DIM; ++aa) Gm[ii][aa] = 0.5 * (xv[aa + 1][ii] - xv[0][ii]);
            double J, inv[DIM][DIM];
            if constexpr (DIM == 2) {
                J = Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0];
                const double iJ = 1.0 / J;
                inv[0][0] = Gm[1][1] * iJ;
                inv[0][1] = -Gm[0][1] * iJ;
                inv[1][0] = -Gm[1][0] * iJ;
                inv[1][1] = Gm[0][0] * iJ;
            } else {
                const double c00 = Gm[1][1] * Gm[2][2] - Gm[1][2] * Gm[2][1];
                const double c01 = Gm[1][2] * Gm[2][0] - Gm[1][0] * Gm[2][2];
                const double c02 = Gm[1][0] * Gm[2][1] - Gm[1][1] * Gm[2][0];
                J = Gm[0][0] * c00 + Gm[0][1] * c01 + Gm[0][2] * c02;
                const double iJ = 1.0 / J;
                inv[0][0] = c00 * iJ;
                inv[1][0] = c01 * iJ;
                inv[2][0] = c02 * iJ;
                inv[0][1] = (Gm[0][2] * Gm[2][1] - Gm[0][1] * Gm[2][2]) * iJ;
                inv[1][1] = (Gm[0][0] * Gm[2][2] - Gm[0][2] * Gm[2][0]) * iJ;
                inv[2][1] = (Gm[0][1] * Gm[2][0] - Gm[0][0] * Gm[2][1]) * iJ;
                inv[0][2] = (Gm[0][1] * Gm[1][2] - Gm[0][2] * Gm[1][1]) * iJ;
                inv[1][2] = (Gm[0][2] * Gm[1][0] - Gm[0][0] * Gm[1][2]) * iJ;
                inv[2][2] = (Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0]) * iJ;
            }
            if (valid && q4 == 0 && !(J > 0.0)) atomicOr(a.err, 1);
#pragma unroll
            for (int aa = 0; aa < DIM; ++aa)
#pragma unroll
                for (int ii = 0; ii < DIM; ++ii) met[aa * DIM + ii] = T(inv[aa][ii]);
            const double halfiJ = 0.5 / J;
            if constexpr (DIM == 2) {
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int va = f, vb = (f + 1) % 3;
                    const double tx = xv[vb][0] - xv[va][0], ty = xv[vb][1] - xv[va][1];
                    const double len = sqrt(tx * tx + ty * ty);
                    const double il = 1.0 / len;
                    nrm[2 * f] = T(ty * il);
                    nrm[2 * f + 1] = T(-tx * il);
                    fsc[f] = T(len * halfiJ);
                }
            } else {
                const int fv[4][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {1, 2, 3, 0}, {0, 2, 3, 1}};
#pragma unroll
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
                    const double inn = 1.0 / nn;
                    nrm[3 * f] = T(n0 * inn);
                    nrm[3 * f + 1] = T(n1 * inn);
                    nrm[3 * f + 2] = T(n2 * inn);
                    fsc[f] = T(0.5 * nn * halfiJ);   // sJ / J with sJ = area / 2 = |n| / 4
                }
            }
#pragma unroll
            for (int v = 0; v < NVERT; ++v)
#pragma unroll
                for (int d = 0; d < DIM; ++d) wvt[v * DIM + d] = T(wv[v][d]);
        }

        V rhs[NRT][NF];
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
            for (int k = 0; k < NF; ++k) rhs[rt][k] = V{T(0), T(0), T(0), T(0)};
        // ---- relaxation source: interpolate, Ntilde, project (tile by tile).
        //      Done first so its density/momentum operands are dead before the
        //      volume term needs registers.
        {
            T bq[NJS][NCONS];
#pragma unroll
            for (int s = 0; s < NJS; ++s) {
                const int j = 4 * s + q4;
#pragma unroll
                for (int kq = 0; kq < NCONS; ++kq) bq[s][kq] = (valid && j < NP) ? own(kq, j) : T(0);
            }
            for (int t = 0; t < nct; ++t) {
                V cc[NCONS];
#pragma unroll
                for (int kq = 0; kq < NCONS; ++kq) cc[kq] = V{T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int s = 0; s < NJS; ++s) {
                    const T afr = s_ops[O::fi(nct, t, s) + lane];
#pragma unroll
                    for (int kq = 0; kq < NCONS; ++kq) cc[kq] = mfma16(afr, bq[s][kq], cc[kq]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pnt = 16 * t + crow<T>(q4, r);
                    T nt[NS];
                    if (valid && pnt < Nc) {
                        T mom[DIM];
#pragma unroll
                        for (int d = 0; d < DIM; ++d) mom[d] = cc[1 + d][r];
                        ntilde<DIM, T>(cc[0][r] + kc.rho0, mom, kc.inv_tau, nt);
                    } else {
#pragma unroll
                        for (int sf = 0; sf < NS; ++sf) nt[sf] = T(0);
                    }
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt) {
                        const T pfr = s_ops[O::fp(nct, rt, t, r) + lane];
#pragma unroll
                        for (int sf = 0; sf < NS; ++sf) rhs[rt][NCONS + sf] = mfma16(pfr, nt[sf], rhs[rt][NCONS + sf]);
                    }
                }
            }
        }

        // ---- volume term, one field at a time
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            V acc[NRT][DIM];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int d = 0; d < DIM; ++d) acc[rt][d] = V{T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int s = 0; s < NJS; ++s) {
                const int j = 4 * s + q4;
                const T b = (valid && j < NP) ? own(k, j) : T(0);
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                    for (int d = 0; d < DIM; ++d) acc[rt][d] = mfma16(s_ops[O::fd(d, rt, s) + lane], b, acc[rt][d]);
            }
            // chain rule, -c M_d scatter and the ALE term w . grad q for this field
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 16 * rt + crow<T>(q4, r);
                    const int ib = (i < NP ? i : 0) * NVERT;
#pragma unroll
                    for (int ii = 0; ii < DIM; ++ii) {
                        T gph = T(0);
#pragma unroll
                        for (int aa = 0; aa < DIM; ++aa) gph += met[aa * DIM + ii] * acc[rt][aa][r];
                        T w = T(0);
#pragma unroll
                        for (int v = 0; v < NVERT; ++v) w += BARY[ib + v] * wvt[v * DIM + ii];
                        rhs[rt][k][r] += w * gph;
#pragma unroll
                        for (int row = 0; row < NF; ++row) {
                            const double mc = mcoef<DIM>(ii, row, k);
                            if (mc != 0.0) rhs[rt][row][r] -= kc.c * T(mc) * gph;
                        }
                    }
                }
        }

        // ---- surface term: upwind flux at this lane's face slots, lifted by
        //      MFMA; the next slot's neighbour values are in flight meanwhile
#pragma unroll 1
        for (int s2 = 0; s2 < NMS; ++s2) {
            const int m = 4 * s2 + q4;
            const int32_t idx = vm_cur;
            T nbv[NF];
#pragma unroll
            for (int k = 0; k < NF; ++k) nbv[k] = nb_cur[k];
            if (s2 + 1 < NMS) {
                gather(s2 + 1, vm_nxt, nb_cur);
                vm_cur = vm_nxt;
                if (s2 + 2 < NMS) vm_nxt = vmg[(s2 + 2) * 64];
            }
            T fl[NF];
#pragma unroll
            for (int k = 0; k < NF; ++k) fl[k] = T(0);
            const int vm = s_slot[2 * m];
            if (valid && vm >= 0) {
                const int f = s_slot[2 * m + 1];
                T y[NF];
                if (idx >= 0) {
#pragma unroll
                    for (int k = 0; k < NF; ++k) y[k] = own(k, vm) - nbv[k];
                } else if (idx == -1) {
#pragma unroll
                    for (int k = 0; k < NF; ++k) y[k] = T(0);
                    const T rho = own(0, vm) + kc.rho0;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) {
                        T wd = T(0);
#pragma unroll
                        for (int v = 0; v < NVERT; ++v) wd += BARY[vm * NVERT + v] * wvt[v * DIM + d];
                        const T mm = own(1 + d, vm);
                        y[1 + d] = mm - (T(2) * rho * wd / kc.c - mm);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NF; ++k) y[k] = own(k, vm) - kc.q_inf[k];
                }
                // normal and sJ/J of this slot's face, selected without dynamic
                // register indexing
                T nv[DIM], fs = T(0), wn = T(0);
#pragma unroll
                for (int d = 0; d < DIM; ++d) nv[d] = T(0);
#pragma unroll
                for (int ff = 0; ff < NFACES; ++ff)
                    if (ff == f) {
#pragma unroll
                        for (int d = 0; d < DIM; ++d) nv[d] = nrm[ff * DIM + d];
                        fs = fsc[ff];
                    }
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    T wd = T(0);
#pragma unroll
                    for (int v = 0; v < NVERT; ++v) wd += BARY[vm * NVERT + v] * wvt[v * DIM + d];
                    wn += wd * nv[d];
                }
                if (kc.flux_mode == 0) {
                    // split upwinding: (c M_n)^- y + min(-w.n, 0) y, the first
                    // part by Horner's scheme in M_n with solver constants
#pragma unroll
                    for (int k = 0; k < NF; ++k) fl[k] = kc.fluxA[4] * y[k];
#pragma unroll
                    for (int p = 3; p >= 0; --p) {
                        T z[NF];
                        apply_Mn<DIM, T>(nv, fl, z);
                        const T ap = p == 0 ? kc.fluxA[0] + tmin(-wn, T(0)) : kc.fluxA[p];
#pragma unroll
                        for (int k = 0; k < NF; ++k) fl[k] = z[k] + ap * y[k];
                    }
                } else {
                    // relative upwinding: weights min(c lambda - w.n, 0) on the
                    // spectrum, turned into polynomial coefficients per node
                    T gl[5];
                    const T cs3 = kc.c * T(1.7320508075688772);
                    const T lam[5] = {-cs3, -kc.c, T(0), kc.c, cs3};
#pragma unroll
                    for (int l = 0; l < 5; ++l) gl[l] = tmin(lam[l] - wn, T(0));
                    T cp = T(0);
#pragma unroll
                    for (int l = 0; l < 5; ++l) cp += kc.fluxV[l] * gl[l];
#pragma unroll
                    for (int k = 0; k < NF; ++k) fl[k] = cp * y[k];
#pragma unroll
                    for (int p = 1; p < 5; ++p) {
                        T z[NF];
                        apply_Mn<DIM, T>(nv, y, z);
                        cp = T(0);
#pragma unroll
                        for (int l = 0; l < 5; ++l) cp += kc.fluxV[p * 5 + l] * gl[l];
#pragma unroll
                        for (int k = 0; k < NF; ++k) {
                            y[k] = z[k];
                            fl[k] += cp * z[k];
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < NF; ++k) fl[k] *= fs;
            }
#pragma unroll
            for (int k = 0; k < NF; ++k)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) rhs[rt][k] = mfma16(s_ops[O::fl(rt, s2) + lane], fl[k], rhs[rt][k]);
        }

        // ---- sponge, SARK-4 stage combination and store (this lane's rows)
        double spx[NVERT][2];
        if constexpr (DIM == 2) {
            if (kc.sponge) {
#pragma unroll
                for (int v = 0; v < NVERT; ++v) {
                    spx[v][0] = a.xs[int64_t(vid[v]) * DIM + 0];
                    spx[v][1] = a.xs[int64_t(vid[v]) * DIM + 1];
                }
            }
        }
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * rt + crow<T>(q4, r);
                if (!valid || i >= NP) continue;
                T rv[NF];
#pragma unroll
                for (int k = 0; k < NF; ++k) rv[k] = rhs[rt][k][r];
                if constexpr (DIM == 2) {
                    if (kc.sponge) {
                        double px = 0.0, py = 0.0;
#pragma unroll
                        for (int v = 0; v < NVERT; ++v) {
                            px += double(BARY[i * NVERT + v]) * spx[v][0];
                            py += double(BARY[i * NVERT + v]) * spx[v][1];
                        }
                        const double rr = sqrt((px - kc.sp_cx) * (px - kc.sp_cx) + (py - kc.sp_cy) * (py - kc.sp_cy));
                        double xi = (rr - kc.sp_r0) / (kc.sp_r1 - kc.sp_r0);
                        xi = xi < 0.0 ? 0.0 : (xi > 1.0 ? 1.0 : xi);
                        const T sig = T(kc.sp_smax * xi * xi);
#pragma unroll
                        for (int k = 0; k < NF; ++k)
                            rv[k] -= sig * (own(k, i) - kc.q_inf[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < NF; ++k) {
                    const StageCoef<T> &cf = kc.cf[k < NCONS ? 0 : 1];
                    const int addr = (k * NP + i) * 16 + col;
                    if constexpr (STAGE == kRhsOnly || STAGE == kStage0) {
                        Aw[addr] = rv[k];
                    } else if constexpr (STAGE == kStage1) {
                        const T qn = Qw[addr], f0 = Aw[addr];
                        Bw[addr] = cf.E2 * qn + cf.a20 * f0 + cf.a21 * rv[k];
                        Gw[addr] = cf.E4 * qn + cf.b0 * f0 + cf.b1 * rv[k];
                    } else if constexpr (STAGE == kStage2) {
                        const T qn = Qw[addr], f0 = Aw[addr], gg = Gw[addr];
                        Aw[addr] = cf.E3 * qn + cf.a30 * f0 + cf.a32 * rv[k];
                        Gw[addr] = gg + cf.b2 * rv[k];
                    } else {
                        const T v = Gw[addr] + cf.b3 * rv[k];
                        Qw[addr] = v;
                        if (k == 0 && !(v + kc.rho0 > T(0))) atomicOr(a.err, 2);
                    }
                }
            }
        // every lane is done with this wave's LDS block before the next group
        // overwrites it
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace gbd
