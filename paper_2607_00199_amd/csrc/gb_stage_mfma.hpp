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

// Sixteen independent 4x4x1 products (v_mfma_f32_4x4x1f32, a quarter of the
// cycles of the 16x16x4 form).  Measured lane layout on gfx950: lane l holds
// A(block l/4, row l%4), B(block l/4, column l%4) and, in slot r, the result
// (block l/4, row r, column l%4).  With block = 4 (l/16) + (l%16)/4 this is
// a 4-row tile over the 16 element columns whose contraction is split four
// ways by lane/16: the B operand is exactly the 16x16x4 form's, and the four
// partial sums of a column are added across lanes l, l+16, l+32, l+48.
__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// Row tiles of the node contractions.  A 16-row tile runs on 16x16x4
// products.  In FP32, a last 16-row tile with at most kThinRows real rows
// (tetrahedra of order 1 and 3, triangles of order 1) is replaced by 4-row
// thin tiles on mfma4: tile rt >= nfull holds rows 16 nfull + 4 (rt - nfull)
// + r in every lane, as four partial sums over the contraction index split
// by lane/16.  Two thin tiles for a last tile of 5 to 8 rows (triangles of
// order 2 and 5) measured slower than one 16-row tile (order 5: 313 ->
// 329 us per stage on the airfoil O-grid): their cross-lane reductions and
// accumulators cost more than the products saved.
constexpr int kThinRows = 4;
__host__ __device__ constexpr int tiles_full(int np, bool f32) {
    return (f32 && np - 16 * ((np + 15) / 16 - 1) <= kThinRows) ? (np + 15) / 16 - 1 : (np + 15) / 16;
}
__host__ __device__ constexpr int tiles_all(int np, bool f32) {
    return tiles_full(np, f32) + (tiles_full(np, f32) == (np + 15) / 16 ? 0 : (np - 16 * tiles_full(np, f32) + 3) / 4);
}
__host__ __device__ constexpr int tile_row0(int rt, int nfull) { return rt < nfull ? 16 * rt : 16 * nfull + 4 * (rt - nfull); }

template <int DIM, int N, typename T>
struct Tiles {
    static constexpr int NFULL = tiles_full(Shape<DIM, N>::NP, sizeof(T) == 4);
    static constexpr int NRT = tiles_all(Shape<DIM, N>::NP, sizeof(T) == 4);
    static constexpr bool THIN = NRT > NFULL;
};

// The last 16-point cubature tile holds at most four real points (FP32; the
// 49-point rule of the order-4 triangle has one): it is interpolated by
// 4x4x1 blocks, lane (q, c) then takes point 16 t + q of element c, and the
// projection over those four points is one 16x16x4 product (fragment slot
// r = 0 holds P(row, 16 t + q); slots 1..3 are unused).
__host__ __device__ constexpr bool thin_cub_tile(int Nc, bool f32) {
    return f32 && Nc - 16 * ((Nc + 15) / 16 - 1) <= 4;
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
//   FD [DIM][NRT][NJS]   lane (q, c): D_a(row(rt, c), 4 s + q)
//   FL [NRT][NMS]        LIFT(row(rt, c), fn(4 s + q))
//   FI [NCT][NJS]        Icub(16 t + c, 4 s + q)
//   FP [NRT][NCT][4]     Pcub(row(rt, c), 16 t + crow(q, r))
//   BARY [NP][NVERT]
// with row(rt, c) = 16 rt + c on a 16-row tile and tile_row0(rt) + c % 4 on a
// thin one (NRT counts both kinds), then an int table SLOT [4 NMS][2]:
// (volume node, face) of face slot m, or -1.  fn(m) is the face node of slot
// m: face m % 4, node m / 4 on tetrahedra, so the lanes of quarter q of an
// element hold face q in every step; the face-node order on triangles.
template <int DIM, int N, typename T>
struct MOps {
    using M = MShape<DIM, N>;
    using S = Shape<DIM, N>;
    static constexpr int NRT = Tiles<DIM, N, T>::NRT;
    __host__ __device__ static constexpr int fd(int a, int rt, int s) { return ((a * NRT + rt) * M::NJS + s) * 64; }
    __host__ __device__ static constexpr int fl(int rt, int s) { return (DIM * NRT * M::NJS + rt * M::NMS + s) * 64; }
    __host__ __device__ static constexpr int fi_base() { return (DIM * NRT * M::NJS + NRT * M::NMS) * 64; }
    __host__ __device__ static int fi(int nct, int t, int s) { (void)nct; return fi_base() + (t * M::NJS + s) * 64; }
    __host__ __device__ static int fp(int nct, int rt, int t, int r) {
        return fi_base() + nct * M::NJS * 64 + ((rt * nct + t) * 4 + r) * 64;
    }
    __host__ __device__ static int bary(int nct) { return fi_base() + nct * M::NJS * 64 + NRT * nct * 4 * 64; }
    __host__ __device__ static int total(int nct) { return bary(nct) + S::NP * S::NVERT; }
    __host__ __device__ static constexpr int slots() { return 4 * M::NMS; }
};

// Workgroup LDS: operator fragments, the slot table, then one stage-input
// block [NF][Np][16] per wavefront (kWaves wavefronts of 64 lanes).
constexpr int kWaves = 4;

template <int DIM, int N, typename T>
__host__ __device__ inline size_t mfma_lds_state_offset(int nct) {
    size_t b = size_t(MOps<DIM, N, T>::total(nct)) * sizeof(T);
    b = (b + 15) / 16 * 16;
    b += size_t(MOps<DIM, N, T>::slots()) * 2 * sizeof(int32_t);
    return (b + 15) / 16 * 16;
}

// The stage-input block is staged in LDS unless the operators already take
// most of it (tetrahedra of order 3 in FP64: about 80 KB of fragments).
template <int DIM, int N, typename T>
__host__ __device__ constexpr bool stage_in_lds() {
    return !(DIM == 3 && N >= 3 && sizeof(T) == 8);
}

// Blocks of the group's state staged per wavefront: two where they fit (the
// stage input and a second array the stage combination needs: q_n in stage
// 1, G in stage 3), one otherwise (triangles of order 5 in FP64: about
// 47 KB of fragments plus 16 KB per block and wavefront).
template <int DIM, int N, typename T>
__host__ __device__ constexpr int stage_lds_arrays() {
    return !stage_in_lds<DIM, N, T>() ? 0 : (sizeof(T) == 8 && DIM == 2 && N >= 5) ? 1 : 2;
}

template <int DIM, int N, typename T>
__host__ __device__ inline size_t mfma_lds_bytes(int nct, int waves = kWaves) {
    using S = Shape<DIM, N>;
    const size_t state = size_t(stage_lds_arrays<DIM, N, T>()) * waves * S::NF * S::NP * 16 * sizeof(T);
    return mfma_lds_state_offset<DIM, N, T>(nct) + state;
}

// Blocked state address of (element e, field k, node j).
template <int NF, int NP>
__device__ __forceinline__ int64_t baddr(int64_t e, int k, int j) {
    return ((((e >> 4) * NF + k) * NP + j) << 4) + (e & 15);
}

// Solver constants are read through the constant address space: a launch
// never writes them, so the compiler may fetch them with scalar loads into
// scalar registers instead of reloading them per lane inside guarded code.
#define GB_CONST __attribute__((address_space(4)))
template <typename T>
using KConstRef = const GB_CONST KConst<T> &;
template <typename T>
__device__ __forceinline__ KConstRef<T> kconst_ref(const KConst<T> *p) {
    return *(const GB_CONST KConst<T> *)p;
}

// Stage input of field k at a blocked offset `off` (relative to the state
// arrays' common base), formed from the resident arrays for the stage being
// evaluated.
template <int NCONS, int STAGE, typename T>
__device__ __forceinline__ T stage_in_at(const T *Q, const T *A, const T *B, KConstRef<T> kc, int k, int64_t off) {
    (void)kc;
    (void)k;
    if constexpr (STAGE == kStage0 || STAGE == kRhsOnly) {
        return Q[off];
    } else if constexpr (STAGE == kStage1) {
        return A[off];   // q_n1, stored by stage 0
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

// Wavefronts per workgroup of the single-mesh stage kernel, which runs one
// workgroup per CU: eight for kernels at two wavefronts per SIMD (measured
// 2.6 % faster on the 2D TGV than two 4-wavefront workgroups per CU), four
// for the others.
template <int DIM, int N, typename T>
__host__ __device__ constexpr int stage_wg_waves() {
    return stage_waves_per_eu<DIM, N>(sizeof(T)) >= 2 ? 2 * kWaves : kWaves;
}

template <int DIM, int N, typename T, int STAGE>
__global__ void __launch_bounds__((64 * stage_wg_waves<DIM, N, T>()))
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<DIM, N>(sizeof(T))))) stage_mfma_kernel(KArgs<T> a) {
    using S = Shape<DIM, N>;
    using MS = MShape<DIM, N>;
    using O = MOps<DIM, N, T>;
    using V = typename Vec4<T>::type;
    constexpr int NP = S::NP, NF = S::NF, NFT = S::NFT, NCONS = S::NCONS, NS = S::NS, NVERT = S::NVERT;
    constexpr int NFACES = S::NFACES, NJS = MS::NJS, NRT = Tiles<DIM, N, T>::NRT, NMS = MS::NMS;
    const int Nc = a.Nc;
    const int nct = (Nc + 15) / 16;

    extern __shared__ __align__(16) unsigned char smem[];
    T *s_ops = reinterpret_cast<T *>(smem);
    const int nops = O::total(nct);
    int32_t *s_slot = reinterpret_cast<int32_t *>(smem + (size_t(nops) * sizeof(T) + 15) / 16 * 16);
    for (int p = threadIdx.x; p < nops; p += blockDim.x) s_ops[p] = a.ops[p];
    for (int p = threadIdx.x; p < 2 * O::slots(); p += blockDim.x) s_slot[p] = a.fmask[p];
    __syncthreads();

    KConstRef<T> kc = kconst_ref(a.kc);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
    const int col = lane & 15;
    const int q4 = lane >> 4;
    const T *BARY = s_ops + O::bary(nct);
    constexpr int BLK = NF * NP * 16;
    T *s_q = reinterpret_cast<T *>(smem + mfma_lds_state_offset<DIM, N, T>(nct)) +
             wave * BLK * stage_lds_arrays<DIM, N, T>();

    int logical = blockIdx.x;
    if ((gridDim.x & 7) == 0) logical = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    // a contiguous range of groups per workgroup, or blocks of nwave
    // consecutive groups dealt to the workgroups round robin
    int g_begin, g_end, g_step;
    if (a.stride > 0) {
        g_begin = logical * nwave;
        g_end = a.nbatch;
        g_step = a.stride * nwave;
    } else {
        g_begin = logical * a.chunk;
        g_end = g_begin + a.chunk < a.nbatch ? g_begin + a.chunk : a.nbatch;
        g_step = nwave;
    }

    // Triangle kernels load the vertex ids and the first two trace-map
    // entries of a wave's next group while the current group computes, so a
    // group's vertex data is requested together with its stage input.
    constexpr bool kPF = DIM == 2;
    int32_t pf_vm[2] = {0, 0};
    int32_t pf_vid[NVERT] = {};
    auto prefetch = [&](int gn) {
        const int32_t *vmn = a.vmapP + int64_t(gn) * (O::slots() * 16) + q4 * 16 + col;
        pf_vm[0] = vmn[0];
        pf_vm[1] = NMS > 1 ? vmn[64] : 0;
        const int64_t en = int64_t(gn) * 16 + col;
#pragma unroll
        for (int v = 0; v < NVERT; ++v) pf_vid[v] = a.etov[(en < a.K ? en : 0) * NVERT + v];
    };
    if (kPF && g_begin + wave < g_end) prefetch(g_begin + wave);

    for (int gi = g_begin + wave; gi < g_end; gi += g_step) {
        const int g = __builtin_amdgcn_readfirstlane(gi);
        const int pf_next = gi + g_step < g_end ? g + g_step : -1;
#include "gb_stage_body.inc"
    }
}

// Request table of the batched stage kernel: one entry per mesh of a class
// (same dimension, order, precision and cubature rule, so one set of operator
// fragments serves every entry).
// Pointers in the table are declared in the global address space (they come
// from hipMalloc), so the kernel reaches the buffers with global rather than
// flat memory instructions.
#define GB_GLOBAL __attribute__((address_space(1)))

template <typename T>
struct BatchEntry {
    int64_t K, nv;
    GB_GLOBAL const int32_t *etov;
    GB_GLOBAL const double *vstage, *wstage;   // [5][nv][DIM], [4][nv][DIM]
    GB_GLOBAL const int32_t *vmapP;
    GB_GLOBAL T *Q, *A, *B, *G;
    GB_GLOBAL const double *clock;             // [t, step]
    GB_GLOBAL const KConst<T> *kc;
    GB_GLOBAL int *err;
    double target;                             // step count at which the request stops
};

template <typename T>
struct BatchArgs {
    const BatchEntry<T> *ent;
    const int32_t *group_begin;      // [nreq]: first group of each entry, ascending
    int nreq;
    int total;                       // groups over all entries
    int chunk;                       // groups per workgroup (contiguous ranges)
    int stride;                      // > 0: workgroups take every stride-th block of waves groups instead
    int Nc;
    const T *ops;
    const int32_t *fmask;
};

// Dynamic LDS of the batched kernel for a workgroup of `waves` wavefronts:
// the single-mesh layout sized for that many wavefronts, then the group
// offsets of the nreq entries.
template <int DIM, int N, typename T>
__host__ __device__ inline size_t batch_lds_bytes(int nct, int nreq, int waves) {
    return (mfma_lds_bytes<DIM, N, T>(nct, waves) + 15) / 16 * 16 + size_t(nreq) * sizeof(int32_t);
}

// Workgroup sizes the batched kernel can run with: four wavefronts, or
// eight where the kernel targets two wavefronts per SIMD (its registers then
// allow eight of them on the four SIMDs of a CU).
template <int DIM, int N, typename T>
__host__ __device__ constexpr int batch_max_waves() {
    return stage_waves_per_eu<DIM, N>(sizeof(T)) >= 2 ? 2 * kWaves : kWaves;
}

// Batched stage kernel (request-table form, see gb.h): the groups of every
// entry of the table form one index space; a workgroup takes a contiguous
// range of it (XCD-aware, as in stage_mfma_kernel), finds each group's entry
// in an LDS copy of the group offsets and runs the same per-group body on
// that entry's buffers.  A request whose step counter has reached its target
// is skipped.  Built only for the shapes whose kernel needs no scratch
// memory (batch_enabled).
template <int DIM, int N, typename T>
__host__ __device__ constexpr bool batch_enabled() {
    return !(sizeof(T) == 8 && (DIM == 3 || N >= 5)) && !(DIM == 3 && N >= 3);
}

template <int DIM, int N, typename T, int STAGE>
__global__ void __launch_bounds__((64 * batch_max_waves<DIM, N, T>()))
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<DIM, N>(sizeof(T)))))
stage_batch_kernel(BatchArgs<T> b, const BatchEntry<T> *__restrict__ ent) {
    using S = Shape<DIM, N>;
    using MS = MShape<DIM, N>;
    using O = MOps<DIM, N, T>;
    using V = typename Vec4<T>::type;
    constexpr int NP = S::NP, NF = S::NF, NCONS = S::NCONS, NS = S::NS, NVERT = S::NVERT;
    constexpr int NFACES = S::NFACES, NJS = MS::NJS, NRT = Tiles<DIM, N, T>::NRT, NMS = MS::NMS;
    const int Nc = b.Nc;
    const int nct = (Nc + 15) / 16;

    extern __shared__ __align__(16) unsigned char smem[];
    T *s_ops = reinterpret_cast<T *>(smem);
    const int nops = O::total(nct);
    int32_t *s_slot = reinterpret_cast<int32_t *>(smem + (size_t(nops) * sizeof(T) + 15) / 16 * 16);
    for (int p = threadIdx.x; p < nops; p += blockDim.x) s_ops[p] = b.ops[p];
    for (int p = threadIdx.x; p < 2 * O::slots(); p += blockDim.x) s_slot[p] = b.fmask[p];
    int32_t *s_gb =
        reinterpret_cast<int32_t *>(smem + (mfma_lds_bytes<DIM, N, T>(nct, int(blockDim.x >> 6)) + 15) / 16 * 16);
    for (int p = threadIdx.x; p < b.nreq; p += blockDim.x) s_gb[p] = b.group_begin[p];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwave = blockDim.x >> 6;
    const int col = lane & 15;
    const int q4 = lane >> 4;
    const T *BARY = s_ops + O::bary(nct);
    constexpr int BLK = NF * NP * 16;
    T *s_q = reinterpret_cast<T *>(smem + mfma_lds_state_offset<DIM, N, T>(nct)) +
             wave * BLK * stage_lds_arrays<DIM, N, T>();

    int logical = blockIdx.x;
    if ((gridDim.x & 7) == 0) logical = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    // a contiguous range of groups per workgroup, or (tuning option) blocks of
    // nwave consecutive groups dealt to the workgroups round robin
    int g_begin, g_end, g_step;
    if (b.stride > 0) {
        g_begin = logical * nwave;
        g_end = b.total;
        g_step = b.stride * nwave;
    } else {
        g_begin = logical * b.chunk;
        g_end = g_begin + b.chunk < b.total ? g_begin + b.chunk : b.total;
        g_step = nwave;
    }

    // As in stage_mfma_kernel, triangle kernels load the vertex ids and the
    // first two trace-map entries of a wave's next group (found in the table,
    // possibly another entry's) while the current group computes; after a
    // skipped group they are loaded at the start of the next one.
    constexpr bool kPF = DIM == 2;
    int32_t pf_vm[2] = {0, 0};
    int32_t pf_vid[NVERT] = {};
    bool pf_ok = false;  // pf_vm and pf_vid hold the current group's entries
    auto prefetch = [&](int gtn) {
        const int rn = __builtin_amdgcn_readfirstlane(table_search(s_gb, b.nreq, gtn));
        const BatchEntry<T> &En = ent[rn];
        const int gn = gtn - s_gb[rn];
        const int32_t *vmn = (const int32_t *)En.vmapP + int64_t(gn) * (O::slots() * 16) + q4 * 16 + col;
        pf_vm[0] = vmn[0];
        pf_vm[1] = NMS > 1 ? vmn[64] : 0;
        const int64_t en = int64_t(gn) * 16 + col;
        const int32_t *et = (const int32_t *)En.etov;
#pragma unroll
        for (int v = 0; v < NVERT; ++v) pf_vid[v] = et[(en < En.K ? en : 0) * NVERT + v];
    };

    for (int gi = g_begin + wave; gi < g_end; gi += g_step) {
        const int gt = __builtin_amdgcn_readfirstlane(gi);
        const int r = __builtin_amdgcn_readfirstlane(table_search(s_gb, b.nreq, gt));
        const BatchEntry<T> &E = ent[r];
        if (E.clock[1] >= E.target) {
            pf_ok = false;
            continue;
        }
        KArgs<T> a;
        a.K = E.K;
        a.nbatch = int((E.K + 15) / 16);
        a.Nc = Nc;
        a.chunk = 0;
        a.etov = (const int32_t *)E.etov;
        const int slot = STAGE == kRhsOnly ? 0 : STAGE;
        a.xs = (const double *)(E.vstage + int64_t(slot) * E.nv * DIM);
        a.ws = (const double *)(E.wstage + int64_t(slot) * E.nv * DIM);
        a.vmapP = (const int32_t *)E.vmapP;
        a.ops = b.ops;
        a.fmask = b.fmask;
        a.Q = (T *)E.Q;
        a.A = (T *)E.A;
        a.B = (T *)E.B;
        a.G = (T *)E.G;
        a.clock = (const double *)E.clock;
        a.kc = (const KConst<T> *)E.kc;
        a.err = (int *)E.err;
        KConstRef<T> kc = kconst_ref(a.kc);
        const int g = gt - s_gb[r];
        if (kPF && !pf_ok) prefetch(gt);
        // table index of this wave's next group (the body prefetches it)
        const int pf_next = gi + g_step < g_end ? gt + g_step : -1;
        pf_ok = pf_next >= 0;
#include "gb_stage_body.inc"
    }
}

}  // namespace gbd
