// Host-side launch of the fused stage kernel for one element shape and
// precision.  Each (dimension, order, precision) is compiled in a translation
// unit of its own (gb_shape_*.hip) so the kernels build in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "gb_stage_mfma.hpp"

namespace gbd {

// Everything a stage launch needs from the solver.
struct LaunchArgs {
    int64_t K = 0;
    int64_t nv = 0;
    int Nc = 0;
    int grid = 1;              // workgroups for a full chip (one per CU)
    bool interleave = false;   // groups dealt to workgroups round robin instead of in ranges
    size_t lds = 0;            // dynamic LDS bytes per workgroup
    const int32_t *etov = nullptr;
    const double *vstage = nullptr;   // [5][nv][dim] stage vertex positions
    const double *wstage = nullptr;   // [4][nv][dim] stage vertex velocities
    const int32_t *vmapP = nullptr;
    const void *ops = nullptr;
    const int32_t *fmask = nullptr;
    void *Q = nullptr, *A = nullptr, *B = nullptr, *G = nullptr;
    const double *clock = nullptr;
    const void *kc = nullptr;
    int *err = nullptr;
};

// One stage launch of the batched form over a request table.
struct BatchLaunch {
    const void *ent = nullptr;         // BatchEntry<T>[nreq] in device memory
    const int32_t *group_begin = nullptr;
    int nreq = 0;
    int64_t total = 0;                 // element groups over all entries
    int Nc = 0;
    int grid = 1;                      // workgroups to aim for
    int waves = kWaves;                // wavefronts per workgroup (batch_waves)
    bool interleave = false;           // groups dealt to workgroups round robin instead of in ranges
    size_t lds = 0;                    // dynamic LDS bytes (batch_lds of nreq and waves)
    const void *ops = nullptr;
    const int32_t *fmask = nullptr;
};

// Builds a graph of kernel nodes, each depending on the previous one (the
// batched form's replayed steps), without stream capture: the graph can be
// built while other threads make HIP calls.
struct GraphAppender {
    hipGraph_t g = nullptr;
    hipGraphNode_t last = nullptr;
    hipError_t add(const void *func, dim3 grid, dim3 block, size_t lds, void **params) {
        hipKernelNodeParams np{};
        np.func = const_cast<void *>(func);
        np.gridDim = grid;
        np.blockDim = block;
        np.sharedMemBytes = unsigned(lds);
        np.kernelParams = params;
        np.extra = nullptr;
        hipGraphNode_t node;
        const hipError_t e = hipGraphAddKernelNode(&node, g, last ? &last : nullptr, last ? 1 : 0, &np);
        if (e == hipSuccess) last = node;
        return e;
    }
};

struct ShapeEntry {
    hipError_t (*stage)(const LaunchArgs &, int kind, hipStream_t);
    size_t (*lds)(int Nc);
    int (*ops_total)(int Nc);
    // batched form; null for the shapes it is not built for
    hipError_t (*batch_stage)(const BatchLaunch &, int kind, hipStream_t);
    hipError_t (*batch_node)(const BatchLaunch &, int kind, GraphAppender &);
    size_t (*batch_lds)(int Nc, int nreq, int waves);
    int batch_waves_max;
    // raises the dynamic-LDS limit of the batched kernels (outside capture)
    hipError_t (*batch_allow_lds)(size_t bytes);
    // largest per-lane scratch of the batched kernels (0 expected)
    hipError_t (*batch_scratch)(size_t *bytes);
};

// Stage kinds 0..3 are the SARK-4 stages, 4 the plain right-hand side.
template <int DIM, int N, typename T>
hipError_t launch_stage(const LaunchArgs &L, int kind, hipStream_t st) {
    KArgs<T> a{};
    a.K = L.K;
    a.nbatch = int((L.K + 15) / 16);          // groups of 16 elements (one per wavefront)
    a.Nc = L.Nc;
    // each workgroup (W wavefronts) takes a contiguous range of groups, or
    // blocks of W groups round robin
    constexpr int W = stage_wg_waves<DIM, N, T>();
    int grid = std::min(L.grid, (a.nbatch + W - 1) / W);
    if (grid >= 8) grid = grid / 8 * 8;
    a.chunk = (a.nbatch + grid - 1) / grid;
    grid = (a.nbatch + a.chunk - 1) / a.chunk;
    // the XCD-major remap needs a multiple of 8; surplus workgroups find no group
    if (grid >= 8 && grid % 8) grid = (grid + 7) / 8 * 8;
    a.stride = L.interleave ? grid : 0;
    a.etov = L.etov;
    {
        const int64_t stride = L.nv * DIM;
        const int slot = kind == 4 ? 0 : kind;
        a.xs = L.vstage + slot * stride;
        a.ws = L.wstage + slot * stride;
    }
    a.vmapP = L.vmapP;
    a.ops = static_cast<const T *>(L.ops);
    a.fmask = L.fmask;
    a.Q = static_cast<T *>(L.Q);
    a.A = static_cast<T *>(L.A);
    a.B = static_cast<T *>(L.B);
    a.G = static_cast<T *>(L.G);
    a.clock = L.clock;
    a.kc = static_cast<const KConst<T> *>(L.kc);
    a.err = L.err;
    const dim3 block(64 * W);
    using K0 = decltype(&stage_mfma_kernel<DIM, N, T, 0>);
    const K0 fns[5] = {&stage_mfma_kernel<DIM, N, T, 0>, &stage_mfma_kernel<DIM, N, T, 1>,
                       &stage_mfma_kernel<DIM, N, T, 2>, &stage_mfma_kernel<DIM, N, T, 3>,
                       &stage_mfma_kernel<DIM, N, T, 4>};
    const K0 fn = fns[kind < 4 ? kind : 4];
    if (L.lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(L.lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(grid), block, L.lds, st, a);
    return hipGetLastError();
}

// Kernel arguments and grid of a batched stage launch.
template <int DIM, int N, typename T>
int batch_launch_config(const BatchLaunch &L, BatchArgs<T> &b) {
    b = BatchArgs<T>{};
    b.ent = static_cast<const BatchEntry<T> *>(L.ent);
    b.group_begin = L.group_begin;
    b.nreq = L.nreq;
    b.total = int(L.total);
    b.Nc = L.Nc;
    b.ops = static_cast<const T *>(L.ops);
    b.fmask = L.fmask;
    const int waves = L.waves;
    int grid = int(std::min<int64_t>(L.grid, (L.total + waves - 1) / waves));
    if (grid < 1) grid = 1;
    if (grid >= 8) grid = grid / 8 * 8;
    b.chunk = int((L.total + grid - 1) / grid);
    grid = int((L.total + b.chunk - 1) / b.chunk);
    if (grid >= 8 && grid % 8) grid = (grid + 7) / 8 * 8;
    b.stride = 0;
    if (L.interleave) {
        // every workgroup starts at its own index and strides by the grid
        b.chunk = 1;
        b.stride = grid;
    }
    return grid;
}

template <int DIM, int N, typename T>
hipError_t launch_stage_batch(const BatchLaunch &L, int kind, hipStream_t st) {
    BatchArgs<T> b;
    const int grid = batch_launch_config<DIM, N, T>(L, b);
    using K0 = decltype(&stage_batch_kernel<DIM, N, T, 0>);
    const K0 fns[5] = {&stage_batch_kernel<DIM, N, T, 0>, &stage_batch_kernel<DIM, N, T, 1>,
                       &stage_batch_kernel<DIM, N, T, 2>, &stage_batch_kernel<DIM, N, T, 3>,
                       &stage_batch_kernel<DIM, N, T, 4>};
    hipLaunchKernelGGL(fns[kind < 4 ? kind : 4], dim3(grid), dim3(64 * L.waves), L.lds, st, b, b.ent);
    return hipGetLastError();
}

template <int DIM, int N, typename T>
hipError_t node_stage_batch(const BatchLaunch &L, int kind, GraphAppender &ga) {
    BatchArgs<T> b;
    const int grid = batch_launch_config<DIM, N, T>(L, b);
    const BatchEntry<T> *ent = b.ent;
    const void *fns[5] = {(const void *)&stage_batch_kernel<DIM, N, T, 0>, (const void *)&stage_batch_kernel<DIM, N, T, 1>,
                          (const void *)&stage_batch_kernel<DIM, N, T, 2>, (const void *)&stage_batch_kernel<DIM, N, T, 3>,
                          (const void *)&stage_batch_kernel<DIM, N, T, 4>};
    void *params[2] = {&b, &ent};
    return ga.add(fns[kind < 4 ? kind : 4], dim3(grid), dim3(64 * L.waves), L.lds, params);
}

template <int DIM, int N, typename T>
void batch_kernels(const void *out[5]) {
    out[0] = (const void *)&stage_batch_kernel<DIM, N, T, 0>;
    out[1] = (const void *)&stage_batch_kernel<DIM, N, T, 1>;
    out[2] = (const void *)&stage_batch_kernel<DIM, N, T, 2>;
    out[3] = (const void *)&stage_batch_kernel<DIM, N, T, 3>;
    out[4] = (const void *)&stage_batch_kernel<DIM, N, T, 4>;
}

template <int DIM, int N, typename T>
hipError_t batch_allow_lds(size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    const void *fns[5];
    batch_kernels<DIM, N, T>(fns);
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int DIM, int N, typename T>
hipError_t batch_scratch(size_t *bytes) {
    const void *fns[5];
    batch_kernels<DIM, N, T>(fns);
    *bytes = 0;
    for (const void *f : fns) {
        hipFuncAttributes attr;
        hipError_t e = hipFuncGetAttributes(&attr, f);
        if (e != hipSuccess) return e;
        *bytes = std::max(*bytes, size_t(attr.localSizeBytes));
    }
    return hipSuccess;
}

template <int DIM, int N, typename T>
size_t stage_batch_lds(int Nc, int nreq, int waves) { return batch_lds_bytes<DIM, N, T>((Nc + 15) / 16, nreq, waves); }

template <int DIM, int N, typename T>
size_t stage_lds(int Nc) { return mfma_lds_bytes<DIM, N, T>((Nc + 15) / 16, stage_wg_waves<DIM, N, T>()); }

template <int DIM, int N, typename T>
int stage_ops_total(int Nc) { return MOps<DIM, N, T>::total((Nc + 15) / 16); }

template <int DIM, int N, typename T>
ShapeEntry shape_entry() {
    ShapeEntry s{&launch_stage<DIM, N, T>, &stage_lds<DIM, N, T>, &stage_ops_total<DIM, N, T>, nullptr, nullptr, nullptr, 0,
                 nullptr, nullptr};
    if constexpr (batch_enabled<DIM, N, T>()) {
        s.batch_stage = &launch_stage_batch<DIM, N, T>;
        s.batch_node = &node_stage_batch<DIM, N, T>;
        s.batch_lds = &stage_batch_lds<DIM, N, T>;
        s.batch_waves_max = batch_max_waves<DIM, N, T>();
        s.batch_allow_lds = &batch_allow_lds<DIM, N, T>;
        s.batch_scratch = &batch_scratch<DIM, N, T>;
    }
    return s;
}

}  // namespace gbd

#define GB_SHAPE_NAME(D, NN, P) shape_##D##_##NN##_##P
#define GB_DECLARE_SHAPE(D, NN, P) namespace gbd { ShapeEntry GB_SHAPE_NAME(D, NN, P)(); }
#define GB_DEFINE_SHAPE(D, NN, P, TYPE) \
    namespace gbd { ShapeEntry GB_SHAPE_NAME(D, NN, P)() { return shape_entry<D, NN, TYPE>(); } }

#define GB_ALL_SHAPES(X) \
    X(2, 1, f32) X(2, 1, f64) X(2, 2, f32) X(2, 2, f64) X(2, 3, f32) X(2, 3, f64) \
    X(2, 4, f32) X(2, 4, f64) X(2, 5, f32) X(2, 5, f64) \
    X(3, 1, f32) X(3, 1, f64) X(3, 2, f32) X(3, 2, f64) X(3, 3, f32) X(3, 3, f64)
