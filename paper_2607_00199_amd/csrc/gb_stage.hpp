// Shared definitions of the ALE Galerkin-Boltzmann stage kernels: stage kinds,
// SARK-4 stage coefficients, per-solver constants, kernel arguments, element
// shapes, and the per-vertex motion kernels of a step.
//
// A stage evaluates, for every element, the semi-discrete right-hand side F(q)
// of Section 3 (eq. semi_discrete_form, without the stiff -Lambda q part that
// Section 4 integrates exactly) at the geometry of one Runge-Kutta stage and
// stores that stage's SARK-4 combination:
//   geometry  vertex positions of the stage and the grid velocity (Section 5)
//             -> affine metrics, J, outward normals and sJ/J in FP64
//   volume    -c sum_d M_d d_d q + w . grad q  (eq. ale_bns)
//   surface   LIFT [ sJ/J  B~-(q- - q+) ]  (eq. upwind_flux)
//   source    P Ntilde(I q) on the stress fields (cubature)
//   update    the stage's SARK combination (four resident state arrays)
// Upwinding: M_n (normal flux pattern) has spectrum in {-sqrt3,-1,0,1,sqrt3}
// for every unit normal (2D and the 3D tensor system), so the upwind matrix is
// B~- = sum_lambda g(lambda) P_lambda.  Split: g(lambda) = min(c lambda, 0) +
// min(-w.n, 0), with the two negative eigenspaces spanned by explicit
// eigenvectors.  Relative: g(lambda) = min(c lambda - w.n, 0), applied as the
// degree-4 polynomial in M_n that interpolates g on those five points.
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
    // Stage 0 stores q_n1 = E1 q_n + a10 F0 in place of F0, so the later
    // combinations take a10 F0 = q_n1 - E1 q_n with the weights divided by
    // a10: q_n2 = E2 q_n + r20 (q_n1 - E1 q_n) + a21 F1, likewise G (rb0) and
    // q_n3 (r30).  q_n keeps its exact weight E (1 for the density class, so
    // no bias accumulates in FP32), and the difference is of the size of the
    // increment.
    T r20, rb0, r30;
};

// Per-solver constants that change only with dt; kept in device memory and
// read through uniform loads.
template <typename T>
struct KConst {
    StageCoef<T> cf[2];  // [0] density/momentum (no relaxation), [1] stresses
    T c, inv_c, inv_tau, rho0;
    int flux_mode;       // 0 split, 1 relative
    T fluxV[25];         // relative mode, row p: coefficients of g -> power p of M_n
    T q_inf[10];
    int sponge;
    double sp_cx, sp_cy, sp_r0, sp_r1, sp_smax;
    double dt;
    Motion motion;
};

template <typename T>
struct KArgs {
    int64_t K;
    int nbatch;          // number of 16-element groups, ceil(K / 16)
    int Nc;              // cubature points
    int chunk;           // batches per workgroup
    int stride;          // 0: each workgroup a contiguous range of chunk groups;
                         // else blocks of (wavefronts) groups dealt round robin
    const int32_t *etov;
    const double *xs;    // vertex positions of this stage [nv][DIM]
    const double *ws;    // grid velocity at the vertices for this stage [nv][DIM]
    const int32_t *vmapP;
    const T *ops;        // packed operator fragments (see MOps)
    const int32_t *fmask;  // face-slot table: (volume node, face) per slot
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
};

template <typename T>
__device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

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
// for s = 0..3.  The stage velocities are independent, so the work of a
// vertex is spread over four consecutive lanes, one per stage: lane j
// evaluates w_j, writes it and the stage position that starts from it
// (x_n + c_{j+1} dt w_j for j < 3; lane 0 also writes x_n0), and lane 3 takes
// w_0..w_2 from the other three for x_{n+1}.  All four lanes of a vertex must
// be active; a lane with live false computes and takes part in the exchange
// but stores nothing.
template <int DIM>
__device__ __forceinline__ void motion_vertex_lanes(int64_t v, int j, bool live, int64_t nv, const double *X,
                                                    const double *x, double tn, double dt, const Motion &m,
                                                    double *xs, double *ws) {
    const int64_t st = nv * DIM;
    double Xv[DIM], xn[DIM], w[DIM];
    for (int d = 0; d < DIM; ++d) {
        Xv[d] = X[v * DIM + d];
        xn[d] = x[v * DIM + d];
    }
    if (m.kind == 4) {
        for (int d = 0; d < DIM; ++d) w[d] = m.w[j * st + v * DIM + d];
    } else {
        motion_velocity<DIM>(m, Xv, tn + (j == 0 ? 0.0 : j == 3 ? 1.0 : 0.5) * dt, w);
    }
    const int base = int(threadIdx.x & 63) & ~3;
    double w0[DIM], w1[DIM], w2[DIM];
    for (int d = 0; d < DIM; ++d) {
        w0[d] = __shfl(w[d], base + 0);
        w1[d] = __shfl(w[d], base + 1);
        w2[d] = __shfl(w[d], base + 2);
    }
    if (!live) return;
    for (int d = 0; d < DIM; ++d) {
        const int64_t o = v * DIM + d;
        ws[j * st + o] = w[d];
        if (j == 0) xs[o] = xn[d];
        if (j < 3) xs[(j + 1) * st + o] = xn[d] + (j == 2 ? 1.0 : 0.5) * dt * w[d];
        if (j == 3) xs[4 * st + o] = xn[d] + dt * (w0[d] + 2.0 * w1[d] + 2.0 * w2[d] + w[d]) / 6.0;
    }
}

// One mesh: 4 nv threads in blocks of a multiple of 64; lanes past the last
// vertex compute vertex nv - 1 and store nothing.
template <int DIM>
__global__ void motion_stages_kernel(int64_t nv, const double *X, const double *x, const double *clock, double dt,
                                     Motion m, double *xs, double *ws) {
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t v = tid >> 2;
    const bool live = v < nv;
    motion_vertex_lanes<DIM>(live ? v : nv - 1, int(tid & 3), live, nv, X, x, clock[0], dt, m, xs, ws);
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

// ---------------------------------------------------------------- batched form
//
// Many meshes stepped together: the vertex kernels of a step run over the
// concatenated vertex ranges of every request of one dimension, found through
// a request table.  A request whose step counter has reached its target is
// left alone (its stage launches skip it as well), so a captured one-step
// graph can be replayed while requests finish at different steps.

constexpr int kMaxBatch = 1024;   // requests per table

struct MotionEntry {
    int64_t nv, v_begin;           // vertices, first vertex in the concatenation
    const double *X;               // reference positions [nv][DIM]
    double *x;                     // current positions
    double *clock;                 // [t, step]
    double *vstage, *wstage;       // [5][nv][DIM], [4][nv][DIM]
    double dt, target;             // time step; step count at which the request stops
    Motion m;
};

// Request owning vertex (or group) index i: largest r with begin[r] <= i.
template <typename I>
__device__ __forceinline__ int table_search(const I *begin, int n, I i) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (begin[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int DIM>
__global__ void motion_batch_kernel(const MotionEntry *E, int n, int64_t total) {
    __shared__ int64_t s_vb[kMaxBatch];
    for (int p = threadIdx.x; p < n; p += blockDim.x) s_vb[p] = E[p].v_begin;
    __syncthreads();
    // four lanes per vertex (motion_vertex_lanes); the four lanes of a vertex
    // leave together or not at all
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = tid >> 2;
    if (i >= total) return;
    const MotionEntry &e = E[table_search(s_vb, n, i)];
    if (e.clock[1] >= e.target) return;
    motion_vertex_lanes<DIM>(i - e.v_begin, int(tid & 3), true, e.nv, e.X, e.x, e.clock[0], e.dt, e.m, e.vstage,
                             e.wstage);
}

// x_n <- x_{n+1} for every request (a no-op for finished ones, whose stage
// positions still hold their last end-of-step positions); the first vertex of
// an unfinished request advances its clock.  Only that thread reads or writes
// the clock, so the finished test cannot race with the advance.
template <int DIM>
__global__ void finish_batch_kernel(const MotionEntry *E, int n, int64_t total) {
    __shared__ int64_t s_vb[kMaxBatch];
    for (int p = threadIdx.x; p < n; p += blockDim.x) s_vb[p] = E[p].v_begin;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const MotionEntry &e = E[table_search(s_vb, n, i)];
    const int64_t v = i - e.v_begin;
    const double *xnext = e.vstage + 4 * e.nv * DIM;
    for (int d = 0; d < DIM; ++d) e.x[v * DIM + d] = xnext[v * DIM + d];
    if (v == 0 && e.clock[1] < e.target) {
        e.clock[0] = e.clock[0] + e.dt;
        e.clock[1] = e.clock[1] + 1.0;
    }
}

}  // namespace gbd
