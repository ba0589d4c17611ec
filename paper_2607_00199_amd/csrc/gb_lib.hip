// C ABI of the ALE Galerkin-Boltzmann library: handles, host setup, device
// buffers and kernel launches.  See include/gb.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gb.h"
#include "gb_diag.hpp"
#include "gb_launch.hpp"
#include "host_ref.hpp"

namespace {

thread_local std::string g_err;

gb_status fail(gb_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define GB_HIP(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail(GB_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = n;
        return n ? hipMalloc(&p, n) : hipSuccess;
    }
    template <typename U>
    U *as() const { return static_cast<U *>(p); }
};

}  // namespace

// Device scratch for the allocation-free energy diagnostic: per-workgroup
// partial sums and the result.  Every device holds its own copy for the life
// of the process; host code reaches it only through the address returned by
// hipGetSymbolAddress for that device (kept in scratch_addr below).
constexpr size_t kScratchDoubles = 8192;   // 64 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

struct gb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    size_t max_lds = 65536;
    std::string arch;               // gcnArchName, part of the tuning-cache key
    double *scratch = nullptr;      // this device's copy of the scratch array
};

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_addr;   // device -> address of its scratch

// Address of the scratch array on `device` (current device), looked up once
// per device.
hipError_t scratch_addr(int device, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = static_cast<double *>(p);
    *out = static_cast<double *>(p);
    return hipSuccess;
}
}  // namespace

struct gb_mesh {
    gb_ctx *ctx = nullptr;
    int dim = 2, N = 1;
    int64_t K = 0, nv = 0;
    gbh::RefElement ref;            // with the default cubature degree
    gbh::Connectivity conn;
    std::vector<double> X;          // reference vertex positions (host)
    DevBuf d_etov, d_X, d_x, d_vmapP;
    DevBuf d_wv;                    // vertex-array motion: [4][nv][dim] velocities
    DevBuf d_wall;                  // wall faces, element * Nfaces + face
    DevBuf d_fmask, d_wface;        // face node lists [Nfaces][Nfp] and their face-integral weights
    int nwall = 0;
    gbd::Motion motion{};
    int64_t motion_serial = 0;      // bumped by every gb_set_motion
    int solvers = 0;
};

struct gb_solver {
    gb_mesh *mesh = nullptr;
    gb_params prm{};
    gbh::RefElement ref;            // with the solver's cubature degree
    int NF = 6;
    size_t elem_bytes = 4;
    DevBuf Q, A, B, G;              // the four resident arrays
    DevBuf ops, fmask, clock, err;
    DevBuf vstage, wstage;          // per-stage vertex positions [5][nv][dim] and velocities [4][nv][dim]
    DevBuf kconst;                  // gbd::KConst<T> for the current dt
    DevBuf d_icub, d_wcub;          // cubature interpolation [Nc][Np] and weights [Nc], FP64 (diagnostics)
    DevBuf diag;                    // energy reduction: per-workgroup partial sums, then the result
    std::vector<unsigned char> kconst_host;
    double kconst_dt = -1.0;
    int64_t kconst_motion_serial = -1;
    double t = 0.0;
    int64_t step = 0;
    bool has_state = false;
    bool in_batch = false;          // a batch member: stepped and read only through its batch
    int grid = 1;
    bool interleave = false;        // stage launches deal groups round robin instead of in ranges
    size_t lds = 0;
    // timing: an event pair around every stage launch, resolved on query
    bool timing = false;
    std::vector<hipEvent_t> ev;     // start, stop, start, stop, ...
    std::vector<int> ev_kind;
    double time_ms = 0.0, time_ms_kind[4] = {0, 0, 0, 0};
    int64_t time_launches = 0, launches_kind[4] = {0, 0, 0, 0};
    // graph
    hipGraphExec_t graph_exec = nullptr;
    double graph_dt = 0.0;
    int64_t graph_motion_serial = -1;
    ~gb_solver() {
        for (auto e : ev) (void)hipEventDestroy(e);
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    }
};

namespace {

// ---------------------------------------------------------------- dispatch

struct Launcher {
    gbd::ShapeEntry shape{};
    hipError_t (*prepare)(gb_solver *s, double dt, hipStream_t st) = nullptr;
    // launches one stage kind (0..3 SARK-4 stages, 4 right-hand side only)
    hipError_t stage(gb_solver *s, int kind, double dt, hipStream_t st) const;
    size_t lds(int Nc) const { return shape.lds(Nc); }
    int ops_total(int Nc) const { return shape.ops_total(Nc); }
};

template <typename T>
void fill_coef(gbd::StageCoef<T> &c, const gbh::SarkCoef &h, double dt) {
    c.E1 = T(h.E[1]);
    c.E2 = T(h.E[2]);
    c.E3 = T(h.E[3]);
    c.E4 = T(h.E[4]);
    c.a10 = T(dt * h.a10);
    c.a20 = T(dt * h.a20);
    c.a21 = T(dt * h.a21);
    c.a30 = T(dt * h.a30);
    c.a32 = T(dt * h.a32);
    c.b0 = T(dt * h.b[0]);
    c.b1 = T(dt * h.b[1]);
    c.b2 = T(dt * h.b[2]);
    c.b3 = T(dt * h.b[3]);
    // weights of q_n1 - E1 q_n = a10 F0, which replaces F0 (a10 = phi1(c1
    // gamma) / 2 > 0 before the dt factor, which cancels in the ratios)
    c.r20 = T(h.a20 / h.a10);
    c.rb0 = T(h.b[0] / h.a10);
    c.r30 = T(h.a30 / h.a10);
}

// coefficients turning the five eigenvalue weights into powers of M_n:
// inverse of V[l][p] = lambda_l^p on {-sqrt3, -1, 0, 1, sqrt3}
void flux_vinv(double out[25]) {
    const double lam[5] = {-std::sqrt(3.0), -1.0, 0.0, 1.0, std::sqrt(3.0)};
    gbh::Mat V(5, 5);
    for (int l = 0; l < 5; ++l)
        for (int p = 0; p < 5; ++p) V(l, p) = std::pow(lam[l], p);
    const gbh::Mat Vi = gbh::inverse(V);
    for (int p = 0; p < 5; ++p)
        for (int l = 0; l < 5; ++l) out[p * 5 + l] = Vi(p, l);
}

template <typename T>
void fill_kconst(gbd::KConst<T> &k, const gb_solver *s, double dt) {
    std::memset(&k, 0, sizeof(k));
    fill_coef(k.cf[0], gbh::sark_coefficients(0.0), dt);
    fill_coef(k.cf[1], gbh::sark_coefficients(-dt / s->prm.tau), dt);
    k.c = T(s->prm.c);
    k.inv_c = T(1.0 / s->prm.c);
    k.inv_tau = T(1.0 / s->prm.tau);
    const double rho0 = s->prm.precision == GB_FP32 ? s->prm.rho0 : 0.0;
    k.rho0 = T(rho0);
    k.flux_mode = s->prm.flux_mode;
    double fv[25];
    flux_vinv(fv);
    for (int p = 0; p < 25; ++p) k.fluxV[p] = T(fv[p]);
    for (int f = 0; f < 10; ++f) k.q_inf[f] = T(s->prm.q_inf[f] - (f == 0 ? rho0 : 0.0));
    k.sponge = s->prm.sponge_sigma_max > 0.0;
    k.sp_cx = s->prm.sponge_cx;
    k.sp_cy = s->prm.sponge_cy;
    k.sp_r0 = s->prm.sponge_r0;
    k.sp_r1 = s->prm.sponge_r1;
    k.sp_smax = s->prm.sponge_sigma_max;
    k.dt = dt;
    k.motion = s->mesh->motion;
}

// Constants for this dt and motion, uploaded in stream order when they change
// (always outside any graph capture).
template <typename T>
hipError_t prepare_consts(gb_solver *s, double dt, hipStream_t st) {
    gb_mesh *m = s->mesh;
    if (s->kconst_dt == dt && s->kconst_motion_serial == m->motion_serial) return hipSuccess;
    gbd::KConst<T> *hk = reinterpret_cast<gbd::KConst<T> *>(s->kconst_host.data());
    fill_kconst(*hk, s, dt);
    hipError_t e = hipMemcpyAsync(s->kconst.p, hk, sizeof(gbd::KConst<T>), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    s->kconst_dt = dt;
    s->kconst_motion_serial = m->motion_serial;
    return hipSuccess;
}

#define GB_DECL(D, NN, P) GB_DECLARE_SHAPE(D, NN, P)
}  // namespace
GB_ALL_SHAPES(GB_DECL)
namespace {
#undef GB_DECL

bool get_launcher(int dim, int N, int prec, Launcher &L) {
    const bool f64 = prec == GB_FP64;
#define GB_CASE(D, NN, P)                                                  \
    if (dim == D && N == NN && f64 == (#P[1] == '6')) {                  \
        L.shape = gbd::GB_SHAPE_NAME(D, NN, P)();                          \
        L.prepare = f64 ? &prepare_consts<double> : &prepare_consts<float>; \
        return true;                                                       \
    }
    GB_ALL_SHAPES(GB_CASE)
#undef GB_CASE
    return false;
}

// Request-table entry of a solver for the batched form.
template <typename T>
gbd::BatchEntry<T> make_entry(const gb_solver *s, double target) {
    const gb_mesh *m = s->mesh;
    gbd::BatchEntry<T> e{};
    e.K = m->K;
    e.nv = m->nv;
    e.etov = (GB_GLOBAL const int32_t *)m->d_etov.as<int32_t>();
    e.vstage = (GB_GLOBAL const double *)s->vstage.as<double>();
    e.wstage = (GB_GLOBAL const double *)s->wstage.as<double>();
    e.vmapP = (GB_GLOBAL const int32_t *)m->d_vmapP.as<int32_t>();
    e.Q = (GB_GLOBAL T *)s->Q.as<T>();
    e.A = (GB_GLOBAL T *)s->A.as<T>();
    e.B = (GB_GLOBAL T *)s->B.as<T>();
    e.G = (GB_GLOBAL T *)s->G.as<T>();
    e.clock = (GB_GLOBAL const double *)s->clock.as<double>();
    e.kc = (GB_GLOBAL const gbd::KConst<T> *)s->kconst.as<gbd::KConst<T>>();
    e.err = (GB_GLOBAL int *)s->err.as<int>();
    e.target = target;
    return e;
}

hipError_t Launcher::stage(gb_solver *s, int kind, double dt, hipStream_t st) const {
    (void)dt;
    const gb_mesh *m = s->mesh;
    gbd::LaunchArgs a;
    a.K = m->K;
    a.nv = m->nv;
    a.Nc = s->ref.Nc;
    a.grid = s->grid;
    a.interleave = s->interleave;
    a.lds = s->lds;
    a.etov = m->d_etov.as<int32_t>();
    a.vstage = s->vstage.as<double>();
    a.wstage = s->wstage.as<double>();
    a.vmapP = m->d_vmapP.as<int32_t>();
    a.ops = s->ops.p;
    a.fmask = s->fmask.as<int32_t>();
    a.Q = s->Q.p;
    a.A = s->A.p;
    a.B = s->B.p;
    a.G = s->G.p;
    a.clock = s->clock.as<double>();
    a.kc = s->kconst.p;
    a.err = s->err.as<int>();
    return shape.stage(a, kind, st);
}

// ---------------------------------------------------------------- conversion kernels

// host layout [K][NF][NP] (FP64) <-> device blocked layout [K/16][NF][NP][16]
__device__ __forceinline__ int64_t blocked_index(int64_t idx, int NP, int NF) {
    const int64_t j = idx % NP;
    const int64_t k = (idx / NP) % NF;
    const int64_t e = idx / (int64_t(NP) * NF);
    return (((e >> 4) * NF + k) * NP + j) * 16 + (e & 15);
}

template <typename T>
__global__ void to_state_kernel(const double *in, T *out, int64_t n, int NP, int NF, double rho0) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int field = int((idx / NP) % NF);
    out[blocked_index(idx, NP, NF)] = T(field == 0 ? in[idx] - rho0 : in[idx]);
}

template <typename T>
__global__ void from_state_kernel(const T *in, double *out, int64_t n, int NP, int NF, double rho0) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int field = int((idx / NP) % NF);
    const double v = double(in[blocked_index(idx, NP, NF)]);
    out[idx] = field == 0 ? v + rho0 : v;
}

// Operator fragments for the matrix-core stage kernel (layout of gbd::MOps).
template <typename T>
std::vector<T> pack_ops(const gbh::RefElement &R, std::vector<int32_t> &slot_table) {
    const int dim = R.dim, Np = R.Np, NFT = R.Nfaces * R.Nfp, Nc = R.Nc, nvert = dim + 1;
    const bool f32 = sizeof(T) == 4;
    const int NJS = (Np + 3) / 4, NRT = gbd::tiles_all(Np, f32), NMS = (NFT + 3) / 4, nct = (Nc + 15) / 16;
    auto crow = [&](int q, int r) { return f32 ? 4 * q + r : q + 4 * r; };
    std::vector<T> o;
    auto frag = [&](auto val) {
        for (int lane = 0; lane < 64; ++lane) o.push_back(T(val(lane & 15, lane >> 4)));
    };
    auto at = [](const gbh::Mat &M, int i, int j) { return (i < M.rows && j < M.cols) ? M(i, j) : 0.0; };
    // thin node tiles (FP32, the last at most eight rows in tiles of four)
    // are contracted by 4x4x1 blocks: lane (q, c) holds row
    // tile_row0(rt) + c % 4 instead of 16 rt + c
    const int nfull = gbd::tiles_full(Np, f32);
    auto row = [&](int rt, int c) { return rt < nfull ? 16 * rt + c : gbd::tile_row0(rt, nfull) + (c & 3); };
    for (int a = 0; a < dim; ++a)
        for (int rt = 0; rt < NRT; ++rt)
            for (int st = 0; st < NJS; ++st)
                frag([&](int c, int q) { return at(R.D[a], row(rt, c), 4 * st + q); });
    for (int rt = 0; rt < NRT; ++rt)
        for (int st = 0; st < NMS; ++st)
            frag([&](int c, int q) { return at(R.LIFT, row(rt, c), gbh::slot_face_node(R, 4 * st + q)); });
    // a thin last cubature tile (at most four real points, FP32): 4x4x1
    // interpolation rows 16 t + c % 4, projection over points 16 t + q in slot 0
    const bool thin_c = gbd::thin_cub_tile(Nc, f32);
    for (int t = 0; t < nct; ++t)
        for (int st = 0; st < NJS; ++st)
            frag([&](int c, int q) {
                return at(R.Icub, 16 * t + ((thin_c && t == nct - 1) ? (c & 3) : c), 4 * st + q);
            });
    for (int rt = 0; rt < NRT; ++rt)
        for (int t = 0; t < nct; ++t)
            for (int r = 0; r < 4; ++r)
                frag([&](int c, int q) {
                    if (thin_c && t == nct - 1) return r == 0 ? at(R.Pcub, row(rt, c), 16 * t + q) : 0.0;
                    return at(R.Pcub, row(rt, c), 16 * t + crow(q, r));
                });
    for (int i = 0; i < Np; ++i)
        for (int v = 0; v < nvert; ++v) o.push_back(T(R.bary(i, v)));
    slot_table.assign(size_t(4 * NMS) * 2, -1);
    for (int mm = 0; mm < NFT; ++mm) {
        const int fn = gbh::slot_face_node(R, mm);
        slot_table[2 * mm] = R.fmask[fn];
        slot_table[2 * mm + 1] = fn / R.Nfp;
    }
    return o;
}

int n_fields(int dim) { return dim == 2 ? 6 : 10; }

bool supported(int dim, int N) { return (dim == 2 && N >= 1 && N <= 5) || (dim == 3 && N >= 1 && N <= 3); }

gb_status check_error_flag(gb_solver *s) {
    int flag = 0;
    GB_HIP(hipMemcpyAsync(&flag, s->err.p, sizeof(int), hipMemcpyDeviceToHost, s->mesh->ctx->stream));
    GB_HIP(hipStreamSynchronize(s->mesh->ctx->stream));
    if (flag & 1) return fail(GB_ERR_MESH, "an element was inverted (J <= 0) during stepping");
    if (flag & 2) return fail(GB_ERR_NONPHYSICAL, "non-positive or NaN density latched on the device");
    return GB_OK;
}

// Time t0, step 0, vertex positions back at the reference positions, error
// latch cleared (after a new state has been enqueued on the context stream).
gb_status reset_clock_and_positions(gb_solver *s, double t0) {
    gb_mesh *m = s->mesh;
    hipStream_t st = m->ctx->stream;
    double clk[2] = {t0, 0.0};
    GB_HIP(hipMemcpyAsync(s->clock.p, clk, sizeof(clk), hipMemcpyHostToDevice, st));
    GB_HIP(hipMemcpyAsync(m->d_x.p, m->d_X.p, m->d_x.bytes, hipMemcpyDeviceToDevice, st));
    GB_HIP(hipMemsetAsync(s->err.p, 0, sizeof(int), st));
    GB_HIP(hipStreamSynchronize(st));
    s->t = t0;
    s->step = 0;
    s->has_state = true;
    return GB_OK;
}

// Solver constants that do not depend on the step size (flux mode, c, tau,
// far field, sponge, motion): the right-hand-side-only launches read only
// these, so a solver that has not stepped yet gets constants for dt = tau
// (any dt would do) and one that has keeps its step size's coefficients.
hipError_t ensure_consts(gb_solver *s, const Launcher &L, hipStream_t st) {
    const double dt = s->kconst_dt > 0.0 ? s->kconst_dt : s->prm.tau;
    return L.prepare(s, dt, st);
}

hipError_t launch_motion(gb_solver *s, double dt, hipStream_t st) {
    gb_mesh *m = s->mesh;
    const int blk = 256;   // four lanes per vertex
    const unsigned nb = unsigned((4 * m->nv + blk - 1) / blk);
    if (m->dim == 2)
        hipLaunchKernelGGL(gbd::motion_stages_kernel<2>, dim3(nb), dim3(blk), 0, st, m->nv, m->d_X.as<double>(),
                           m->d_x.as<double>(), s->clock.as<double>(), dt, m->motion, s->vstage.as<double>(),
                           s->wstage.as<double>());
    else
        hipLaunchKernelGGL(gbd::motion_stages_kernel<3>, dim3(nb), dim3(blk), 0, st, m->nv, m->d_X.as<double>(),
                           m->d_x.as<double>(), s->clock.as<double>(), dt, m->motion, s->vstage.as<double>(),
                           s->wstage.as<double>());
    return hipGetLastError();
}

gb_status enqueue_step(gb_solver *s, const Launcher &L, double dt, hipStream_t st) {
    gb_mesh *m = s->mesh;
    GB_HIP(launch_motion(s, dt, st));
    for (int kind = 0; kind < 4; ++kind) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (s->timing) {
            GB_HIP(hipEventCreate(&e0));
            GB_HIP(hipEventCreate(&e1));
            s->ev.push_back(e0);
            s->ev.push_back(e1);
            s->ev_kind.push_back(kind);
            GB_HIP(hipEventRecord(e0, st));
        }
        GB_HIP(L.stage(s, kind, dt, st));
        if (s->timing) GB_HIP(hipEventRecord(e1, st));
    }
    const int blk = 256;
    const unsigned nb = unsigned((m->nv + blk - 1) / blk);
    const double *xnext = s->vstage.as<double>() + 4 * m->nv * m->dim;
    if (m->dim == 2)
        hipLaunchKernelGGL(gbd::finish_step_kernel<2>, dim3(nb), dim3(blk), 0, st, m->nv, m->d_x.as<double>(), xnext,
                           s->clock.as<double>(), dt);
    else
        hipLaunchKernelGGL(gbd::finish_step_kernel<3>, dim3(nb), dim3(blk), 0, st, m->nv, m->d_x.as<double>(), xnext,
                           s->clock.as<double>(), dt);
    GB_HIP(hipGetLastError());
    return GB_OK;
}

}  // namespace

// ================================================================= batched form

struct gb_batch {
    gb_ctx *ctx = nullptr;
    size_t budget = 0, used = 0;
    uint64_t next_ticket = 1;
    bool autotune = true;
    struct Member {
        gb_solver *s = nullptr;
        double dt = 0.0;
        double target = 0.0;        // step count at which the member stops
        uint64_t ticket = 0;
        size_t bytes = 0;
    };
    std::vector<Member> members;
    struct Class {
        int dim = 2, N = 1, prec = 0, Nc = 0;
        bool solo = false;          // one large member stepped on its own
        std::vector<int> idx;       // member indices
        gbd::ShapeEntry shape{};
        DevBuf ent, gbeg;
        int nreq = 0;
        int64_t total = 0;          // element groups
        size_t lds = 0;
        int grid = 0;
        int waves = gbd::kWaves;    // wavefronts per workgroup
        bool interleave = false;    // groups dealt round robin instead of in ranges
        int vset = -1;              // its vertex subset (solo classes)
        const void *ops = nullptr;
        const int32_t *fmask = nullptr;
    };
    std::vector<Class> classes;
    // vertex tables (gbd::MotionEntry), one subset per large member and one
    // per dimension for the small members, stored back to back in `mot`
    struct VertexSet {
        int dim = 2, first = 0, n = 0;
        int64_t vtot = 0;
    };
    DevBuf mot;
    std::vector<VertexSet> vsets;
    int vsmall[2] = {-1, -1};
    int graph_steps = 0;            // steps held by the captured graph
    hipGraphExec_t graph = nullptr;
    bool dirty = true;
    // members stepped on their own run on these library-owned streams
    // (default priority), up to `concurrency` at a time, so that one member's
    // kernel tails overlap another's; each run forks them from the batch's
    // stream and joins them back into it
    int concurrency = 1;
    std::vector<hipStream_t> aux;
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    ~gb_batch() {
        if (graph) (void)hipGraphExecDestroy(graph);
        for (auto e : join_ev) (void)hipEventDestroy(e);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        for (auto st : aux) (void)hipStreamDestroy(st);
    }
};

namespace {

// Element groups from which a member is stepped on its own (2048 groups of
// 16 elements give one group to each wavefront of two workgroups per CU).
constexpr int64_t kSoloGroups = 2048;

// Launch tile of a batched class: workgroups, wavefronts per workgroup and
// the group-to-workgroup mapping, chosen by timing (tune_class) and kept in a
// process-wide cache keyed by device architecture, shape, precision,
// cubature size, solo/shared and the power-of-two bucket of the element
// groups; the cache can be saved to and loaded from a text file.
struct Tile {
    int grid = 0, waves = gbd::kWaves, interleave = 0;
};
std::mutex g_tile_mu;
std::map<std::string, Tile> g_tiles;

std::string tile_key(const gb_ctx *ctx, const gb_batch::Class &c) {
    int bucket = 0;
    while ((int64_t(2) << bucket) <= c.total) ++bucket;
    return ctx->arch + " " + std::to_string(c.dim) + " " + std::to_string(c.N) + " " + std::to_string(c.prec) + " " +
           std::to_string(c.Nc) + " " + std::to_string(c.solo ? 1 : 0) + " " + std::to_string(bucket);
}

size_t mesh_bytes(const gb_mesh *m) {
    return m->d_etov.bytes + m->d_X.bytes + m->d_x.bytes + m->d_vmapP.bytes + m->d_wv.bytes;
}

size_t solver_bytes(const gb_mesh *m, const gb_params *p) {
    const size_t es = p->precision == GB_FP32 ? 4 : 8;
    return 4 * size_t((m->K + 15) / 16 * 16) * n_fields(m->dim) * m->ref.Np * es +
           (5 + 4) * size_t(m->nv) * m->dim * sizeof(double);
}

template <typename T>
gb_status upload_class_table(gb_batch *b, gb_batch::Class &c) {
    std::vector<gbd::BatchEntry<T>> ent(c.idx.size());
    std::vector<int32_t> gb(c.idx.size());
    std::vector<gbh::BatchMemberLayout> lay(c.idx.size());
    int64_t g = 0;
    for (size_t i = 0; i < c.idx.size(); ++i) {
        const gb_batch::Member &mb = b->members[size_t(c.idx[i])];
        gb_solver *s = mb.s;
        gb_mesh *m = s->mesh;
        ent[i] = make_entry<T>(s, mb.target);
        gb[i] = int32_t(g);
        g += (m->K + 15) / 16;
        lay[i].K = m->K;
        lay[i].nv = m->nv;
        lay[i].etov_bytes = m->d_etov.bytes;
        lay[i].vstage_bytes = s->vstage.bytes;
        lay[i].wstage_bytes = s->wstage.bytes;
        lay[i].vmap_bytes = m->d_vmapP.bytes;
        lay[i].state_bytes = std::min(std::min(s->Q.bytes, s->A.bytes), std::min(s->B.bytes, s->G.bytes));
    }
    if (g >= (int64_t(1) << 31)) return fail(GB_ERR_UNSUPPORTED, "too many element groups in one class");
    {
        const gb_solver *s0 = b->members[size_t(c.idx[0])].s;
        const std::string bad =
            gbh::check_batch_class(c.dim, s0->ref.Np, s0->NF, s0->ref.Nfaces * s0->ref.Nfp, sizeof(T), lay, gb, g,
                                   gbd::kMaxBatch, c.shape.batch_lds(c.Nc, int(c.idx.size()), gbd::kWaves),
                                   b->ctx->max_lds);
        if (!bad.empty()) return fail(GB_ERR_STATE, "batch table check: " + bad);
    }
    c.total = g;
    if (c.ent.alloc(ent.size() * sizeof(ent[0])) != hipSuccess || c.gbeg.alloc(gb.size() * sizeof(int32_t)) != hipSuccess)
        return fail(GB_ERR_OOM, "batch request table");
    GB_HIP(hipMemcpy(c.ent.p, ent.data(), c.ent.bytes, hipMemcpyHostToDevice));
    GB_HIP(hipMemcpy(c.gbeg.p, gb.data(), c.gbeg.bytes, hipMemcpyHostToDevice));
    return GB_OK;
}

gbd::BatchLaunch class_launch(const gb_batch::Class &c, int grid, int waves, bool interleave) {
    gbd::BatchLaunch L;
    L.ent = c.ent.p;
    L.group_begin = c.gbeg.as<int32_t>();
    L.nreq = c.nreq;
    L.total = c.total;
    L.Nc = c.Nc;
    L.grid = grid;
    L.waves = waves;
    L.interleave = interleave;
    L.lds = c.shape.batch_lds(c.Nc, c.nreq, waves);
    L.ops = c.ops;
    L.fmask = c.fmask;
    return L;
}

hipError_t launch_vertex_batch(gb_batch *b, int set, bool finish, hipStream_t st) {
    if (set < 0) return hipSuccess;
    const gb_batch::VertexSet &vs = b->vsets[size_t(set)];
    if (vs.n == 0) return hipSuccess;
    const int blk = 256;
    // the motion kernel runs four lanes per vertex
    const unsigned nb = unsigned(((finish ? 1 : 4) * vs.vtot + blk - 1) / blk);
    const gbd::MotionEntry *E = b->mot.as<gbd::MotionEntry>() + vs.first;
    if (vs.dim == 2) {
        if (finish)
            hipLaunchKernelGGL(gbd::finish_batch_kernel<2>, dim3(nb), dim3(blk), 0, st, E, vs.n, vs.vtot);
        else
            hipLaunchKernelGGL(gbd::motion_batch_kernel<2>, dim3(nb), dim3(blk), 0, st, E, vs.n, vs.vtot);
    } else {
        if (finish)
            hipLaunchKernelGGL(gbd::finish_batch_kernel<3>, dim3(nb), dim3(blk), 0, st, E, vs.n, vs.vtot);
        else
            hipLaunchKernelGGL(gbd::motion_batch_kernel<3>, dim3(nb), dim3(blk), 0, st, E, vs.n, vs.vtot);
    }
    return hipGetLastError();
}

// The vertex kernel of a set as a node of a graph under construction.
hipError_t node_vertex_batch(gb_batch *b, int set, bool finish, gbd::GraphAppender &ga) {
    if (set < 0) return hipSuccess;
    const gb_batch::VertexSet &vs = b->vsets[size_t(set)];
    if (vs.n == 0) return hipSuccess;
    const int blk = 256;
    const unsigned nb = unsigned(((finish ? 1 : 4) * vs.vtot + blk - 1) / blk);
    const gbd::MotionEntry *E = b->mot.as<gbd::MotionEntry>() + vs.first;
    int n = vs.n;
    int64_t vtot = vs.vtot;
    void *params[3] = {&E, &n, &vtot};
    const void *fn = vs.dim == 2 ? (finish ? (const void *)&gbd::finish_batch_kernel<2> : (const void *)&gbd::motion_batch_kernel<2>)
                                 : (finish ? (const void *)&gbd::finish_batch_kernel<3> : (const void *)&gbd::motion_batch_kernel<3>);
    return ga.add(fn, dim3(nb), dim3(blk), 0, params);
}

// Launch tile of a class: the fastest of the candidate tiles for stage 0
// (workgroups per CU 1..16, four or eight wavefronts per workgroup where the
// kernel allows eight, ranges or round-robin dealing of the groups), each
// timed over three launches on the members' current state (see gb.h: the
// state is not changed).
gb_status tune_class(gb_batch *b, gb_batch::Class &c) {
    hipStream_t st = b->ctx->stream;
    GB_HIP(launch_vertex_batch(b, c.solo ? c.vset : b->vsmall[c.dim - 2], false, st));
    const int mults[5] = {1, 2, 4, 8, 16};
    hipEvent_t e0, e1;
    GB_HIP(hipEventCreate(&e0));
    GB_HIP(hipEventCreate(&e1));
    Tile best{b->ctx->num_cu * 2, gbd::kWaves, 0};
    float best_ms = 1e30f;
    gb_status r = GB_OK;
    for (int waves = gbd::kWaves; waves <= c.shape.batch_waves_max && r == GB_OK; waves *= 2) {
        if (c.shape.batch_lds(c.Nc, c.nreq, waves) > b->ctx->max_lds) continue;
        for (int il = 0; il < 2 && r == GB_OK; ++il)
            for (int mi = 0; mi < 5 && r == GB_OK; ++mi) {
                const int grid = b->ctx->num_cu * mults[mi] * gbd::kWaves / waves;
                if (grid < 1) continue;
                const gbd::BatchLaunch L = class_launch(c, grid, waves, il != 0);
                hipError_t e = c.shape.batch_stage(L, 0, st);
                if (e == hipSuccess) e = hipEventRecord(e0, st);
                for (int k = 0; k < 3 && e == hipSuccess; ++k) e = c.shape.batch_stage(L, 0, st);
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    r = fail(GB_ERR_DEVICE, std::string("batch tuning: ") + hipGetErrorString(e));
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = Tile{grid, waves, il};
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r == GB_OK) {
        c.grid = best.grid;
        c.waves = best.waves;
        c.interleave = best.interleave != 0;
    }
    return r;
}

gb_status batch_rebuild(gb_batch *b) {
    hipStream_t st = b->ctx->stream;
    GB_HIP(hipSetDevice(b->ctx->device));
    GB_HIP(hipStreamSynchronize(st));   // queued replays may still read the old tables
    if (b->graph) {
        GB_HIP(hipGraphExecDestroy(b->graph));
        b->graph = nullptr;
    }
    // Members with enough element groups to fill the GPU on their own are
    // stepped one after another, each with its four stages back to back, so
    // each one's state arrays stay in the last-level cache across its stages;
    // the smaller members of a class share one launch per stage.
    b->classes.clear();
    for (size_t i = 0; i < b->members.size(); ++i) {
        const gb_solver *s = b->members[i].s;
        const int dim = s->mesh->dim, N = s->mesh->N, prec = s->prm.precision, Nc = s->ref.Nc;
        const bool solo = (s->mesh->K + 15) / 16 >= kSoloGroups;
        gb_batch::Class *c = nullptr;
        if (!solo)
            for (auto &cc : b->classes)
                if (!cc.solo && cc.dim == dim && cc.N == N && cc.prec == prec && cc.Nc == Nc) c = &cc;
        if (!c) {
            b->classes.emplace_back();
            c = &b->classes.back();
            c->dim = dim;
            c->N = N;
            c->prec = prec;
            c->Nc = Nc;
            c->solo = solo;
        }
        c->idx.push_back(int(i));
    }
    for (auto &c : b->classes) {
        Launcher L;
        if (!get_launcher(c.dim, c.N, c.prec, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel for a batch class");
        c.shape = L.shape;
        c.nreq = int(c.idx.size());
        if (c.nreq > gbd::kMaxBatch) return fail(GB_ERR_UNSUPPORTED, "too many members in one class");
        const gb_status r = c.prec == GB_FP64 ? upload_class_table<double>(b, c) : upload_class_table<float>(b, c);
        if (r != GB_OK) return r;
        c.lds = c.shape.batch_lds(c.Nc, c.nreq, gbd::kWaves);
        if (c.lds > b->ctx->max_lds) return fail(GB_ERR_UNSUPPORTED, "batch class exceeds the LDS of one workgroup");
        // the dynamic-LDS limit of the kernels covers the largest workgroup tried
        size_t lds_max = c.lds;
        for (int w = 2 * gbd::kWaves; w <= c.shape.batch_waves_max; w *= 2) {
            const size_t l = c.shape.batch_lds(c.Nc, c.nreq, w);
            if (l <= b->ctx->max_lds) lds_max = std::max(lds_max, l);
        }
        GB_HIP(c.shape.batch_allow_lds(lds_max));
        const gb_solver *s0 = b->members[size_t(c.idx[0])].s;
        c.ops = s0->ops.p;
        c.fmask = s0->fmask.as<int32_t>();
        c.grid = b->ctx->num_cu * 2;
        c.waves = gbd::kWaves;
        c.interleave = false;
        {
            std::lock_guard<std::mutex> lk(g_tile_mu);
            auto it = g_tiles.find(tile_key(b->ctx, c));
            // a cached tile this kernel cannot run (workgroup too large for its
            // registers or for the LDS) is ignored
            if (it != g_tiles.end() && it->second.waves <= c.shape.batch_waves_max &&
                c.shape.batch_lds(c.Nc, c.nreq, it->second.waves) <= b->ctx->max_lds) {
                c.grid = it->second.grid;
                c.waves = it->second.waves;
                c.interleave = it->second.interleave != 0;
            }
        }
        c.lds = c.shape.batch_lds(c.Nc, c.nreq, c.waves);
    }
    {
        std::vector<gbd::MotionEntry> E;
        b->vsets.clear();
        auto entry = [&](const gb_batch::Member &mb, int64_t v0) {
            const gb_solver *s = mb.s;
            const gb_mesh *m = s->mesh;
            gbd::MotionEntry e{};
            e.nv = m->nv;
            e.v_begin = v0;
            e.X = m->d_X.as<double>();
            e.x = m->d_x.as<double>();
            e.clock = s->clock.as<double>();
            e.vstage = s->vstage.as<double>();
            e.wstage = s->wstage.as<double>();
            e.dt = mb.dt;
            e.target = mb.target;
            e.m = m->motion;
            return e;
        };
        for (auto &c : b->classes) {
            if (!c.solo) continue;
            const gb_batch::Member &mb = b->members[size_t(c.idx[0])];
            gb_batch::VertexSet vs;
            vs.dim = c.dim;
            vs.first = int(E.size());
            vs.n = 1;
            vs.vtot = mb.s->mesh->nv;
            E.push_back(entry(mb, 0));
            c.vset = int(b->vsets.size());
            b->vsets.push_back(vs);
        }
        for (int di = 0; di < 2; ++di) {
            b->vsmall[di] = -1;
            gb_batch::VertexSet vs;
            vs.dim = di + 2;
            vs.first = int(E.size());
            for (const auto &c : b->classes) {
                if (c.solo || c.dim != di + 2) continue;
                for (int i : c.idx) {
                    const gb_batch::Member &mb = b->members[size_t(i)];
                    E.push_back(entry(mb, vs.vtot));
                    vs.vtot += mb.s->mesh->nv;
                    ++vs.n;
                }
            }
            if (vs.n > gbd::kMaxBatch) return fail(GB_ERR_UNSUPPORTED, "too many small members of one dimension");
            if (vs.n) {
                b->vsmall[di] = int(b->vsets.size());
                b->vsets.push_back(vs);
            }
        }
        if (!E.empty()) {
            if (b->mot.alloc(E.size() * sizeof(E[0])) != hipSuccess) return fail(GB_ERR_OOM, "vertex tables");
            GB_HIP(hipMemcpy(b->mot.p, E.data(), b->mot.bytes, hipMemcpyHostToDevice));
        }
    }
    if (b->autotune)
        for (auto &c : b->classes) {
            const std::string key = tile_key(b->ctx, c);
            {
                std::lock_guard<std::mutex> lk(g_tile_mu);
                if (g_tiles.count(key)) continue;
            }
            const gb_status r = tune_class(b, c);
            if (r != GB_OK) return r;
            c.lds = c.shape.batch_lds(c.Nc, c.nreq, c.waves);
            std::lock_guard<std::mutex> lk(g_tile_mu);
            g_tiles[key] = Tile{c.grid, c.waves, c.interleave ? 1 : 0};
        }
    b->dirty = false;
    b->graph_steps = 0;
    return GB_OK;
}

// `steps` steps of every large member (motion, four stages, end of step),
// launched directly: a member whose state fits the last-level cache keeps it
// there from step to step, and its kernels are long enough that launch
// overhead does not matter.  With concurrency > 1 the members are dealt to
// the auxiliary streams round robin (a member always to the same stream, so
// its steps stay ordered); otherwise they run in turn on `st`.
hipError_t batch_launch_solo(gb_batch *b, int steps, hipStream_t st, int use) {
    hipError_t le = hipSuccess;
    int n = 0;
    for (auto &c : b->classes) {
        if (!c.solo) continue;
        hipStream_t cs = use > 1 ? b->aux[size_t(n++ % use)] : st;
        for (int k = 0; k < steps && le == hipSuccess; ++k) {
            le = launch_vertex_batch(b, c.vset, false, cs);
            for (int kind = 0; kind < 4 && le == hipSuccess; ++kind)
                le = c.shape.batch_stage(class_launch(c, c.grid, c.waves, c.interleave), kind, cs);
            if (le == hipSuccess) le = launch_vertex_batch(b, c.vset, true, cs);
        }
    }
    return le;
}

int solo_count(const gb_batch *b) {
    int n = 0;
    for (const auto &c : b->classes) n += c.solo ? 1 : 0;
    return n;
}

// Auxiliary streams for concurrency > 1 (created once, kept for the batch).
gb_status ensure_aux(gb_batch *b) {
    const int want = b->concurrency > 1 ? std::min(b->concurrency, solo_count(b)) : 0;
    if (want <= 1) return GB_OK;
    if (!b->fork_ev) GB_HIP(hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
    while (int(b->aux.size()) < want) {
        hipStream_t st;
        GB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->aux.push_back(st);
        hipEvent_t e;
        GB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->join_ev.push_back(e);
    }
    return GB_OK;
}

bool has_small(const gb_batch *b) {
    for (const auto &c : b->classes)
        if (!c.solo) return true;
    return false;
}

// The graph of `steps` steps of the small members (one launch per class and
// stage), built node by node (no stream capture, so other threads may make
// HIP calls meanwhile, e.g. a served loop's setup worker).
gb_status batch_capture(gb_batch *b, int steps) {
    if (b->graph) {
        GB_HIP(hipGraphExecDestroy(b->graph));
        b->graph = nullptr;
    }
    hipGraph_t g;
    GB_HIP(hipGraphCreate(&g, 0));
    gbd::GraphAppender ga;
    ga.g = g;
    hipError_t e = hipSuccess;
    for (int k = 0; k < steps && e == hipSuccess; ++k) {
        for (int di = 0; di < 2 && e == hipSuccess; ++di) e = node_vertex_batch(b, b->vsmall[di], false, ga);
        for (int kind = 0; kind < 4 && e == hipSuccess; ++kind)
            for (auto &c : b->classes)
                if (e == hipSuccess && !c.solo)
                    e = c.shape.batch_node(class_launch(c, c.grid, c.waves, c.interleave), kind, ga);
        for (int di = 0; di < 2 && e == hipSuccess; ++di) e = node_vertex_batch(b, b->vsmall[di], true, ga);
    }
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(GB_ERR_DEVICE, std::string("batch graph build: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(GB_ERR_DEVICE, std::string("batch graph instantiate: ") + hipGetErrorString(e));
    b->graph_steps = steps;
    return GB_OK;
}

}  // namespace

// ================================================================= C ABI

extern "C" {

const char *gb_last_error(void) { return g_err.c_str(); }

const char *gb_version(void) { return "gb-ale-mi355x 0.1 (gfx950)"; }

gb_status gb_ctx_create(int device, void *stream, gb_ctx **out) {
    if (!out) return fail(GB_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    GB_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(GB_ERR_ARG, "device index out of range");
    GB_HIP(hipSetDevice(device));
    auto c = std::make_unique<gb_ctx>();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    hipDeviceProp_t prop;
    GB_HIP(hipGetDeviceProperties(&prop, device));
    c->num_cu = prop.multiProcessorCount;
    c->max_lds = prop.sharedMemPerBlock;
    c->arch = prop.gcnArchName;
    for (char &ch : c->arch)
        if (ch == ' ' || ch == ':') ch = '_';
    GB_HIP(scratch_addr(device, &c->scratch));
    *out = c.release();
    return GB_OK;
}

void gb_ctx_destroy(gb_ctx *ctx) { delete ctx; }

gb_status gb_stream_create(int device, void **stream) {
    if (!stream) return fail(GB_ERR_ARG, "stream is NULL");
    *stream = nullptr;
    int n = 0;
    GB_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(GB_ERR_ARG, "device index out of range");
    GB_HIP(hipSetDevice(device));
    hipStream_t st;
    GB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    *stream = st;
    return GB_OK;
}

void gb_stream_destroy(void *stream) {
    if (stream) (void)hipStreamDestroy(static_cast<hipStream_t>(stream));
}

gb_status gb_ctx_synchronize(gb_ctx *ctx) {
    if (!ctx) return fail(GB_ERR_ARG, "ctx is NULL");
    GB_HIP(hipStreamSynchronize(ctx->stream));
    return GB_OK;
}

gb_status gb_ref_operator(int dim, int N, int cubature_degree, int which, double *out, int64_t capacity,
                          int64_t *n_out) {
    if (!out || !n_out) return fail(GB_ERR_ARG, "NULL output");
    if (!((dim == 2 && N >= 1 && N <= 8) || (dim == 3 && N >= 1 && N <= 5)))
        return fail(GB_ERR_UNSUPPORTED, "unsupported (dim, N)");
    gbh::RefElement R;
    try {
        R = gbh::build_ref_element(dim, N, cubature_degree);
    } catch (const std::exception &ex) {
        return fail(GB_ERR_ARG, ex.what());
    }
    std::vector<double> v;
    if (which >= 0 && which <= 2) {
        if (which >= dim) return fail(GB_ERR_ARG, "no such derivative for this dimension");
        v = R.D[which].a;
    } else if (which == 3) {
        v = R.LIFT.a;
    } else if (which == 4) {
        v = R.Icub.a;
    } else if (which == 5) {
        v = R.Pcub.a;
    } else if (which == 6) {
        v = R.r;
    } else if (which == 7) {
        v = R.M.a;
    } else {
        return fail(GB_ERR_ARG, "unknown operator id");
    }
    if (int64_t(v.size()) > capacity) return fail(GB_ERR_ARG, "output buffer too small");
    std::memcpy(out, v.data(), v.size() * sizeof(double));
    *n_out = int64_t(v.size());
    return GB_OK;
}

gb_status gb_check_mesh_tables(int dim, int N, int64_t nv, const double *vx, int64_t K, const int32_t *etov,
                               const double *period, const int8_t *face_tag) {
    if (!vx || !etov) return fail(GB_ERR_ARG, "NULL argument");
    if (dim != 2 && dim != 3) return fail(GB_ERR_ARG, "dim must be 2 or 3");
    if (!supported(dim, N)) return fail(GB_ERR_UNSUPPORTED, "polynomial order not built for this dimension");
    if (nv <= 0 || K <= 0) return fail(GB_ERR_ARG, "empty mesh");
    try {
        const gbh::RefElement ref = gbh::build_ref_element(dim, N, 0);
        std::string err;
        const gbh::Connectivity conn = gbh::build_connectivity(ref, nv, vx, K, etov, period, face_tag, err);
        if (!err.empty()) return fail(GB_ERR_MESH, err);
        const std::vector<int32_t> blk = gbh::blocked_trace_map(ref, K, conn);
        const std::string bad = gbh::check_mesh_tables(ref, nv, K, etov, conn, blk);
        if (!bad.empty()) return fail(GB_ERR_MESH, bad);
    } catch (const std::exception &ex) {
        return fail(GB_ERR_ARG, ex.what());
    }
    return GB_OK;
}

gb_status gb_check_batch_layout(int dim, int N, int precision, int cubature_degree, int nmembers, const int64_t *K,
                                const int64_t *nv, size_t lds_limit, size_t *lds_bytes) {
    if (!K || !nv || !lds_bytes || nmembers <= 0) return fail(GB_ERR_ARG, "NULL argument or no member");
    Launcher L;
    if (!get_launcher(dim, N, precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel for this shape");
    try {
        const gbh::RefElement ref = gbh::build_ref_element(dim, N, cubature_degree);
        const size_t es = precision == GB_FP32 ? 4 : 8;
        const int NF = n_fields(dim), NFT = ref.Nfaces * ref.Nfp, slots = (NFT + 3) / 4 * 4;
        std::vector<gbh::BatchMemberLayout> lay(static_cast<size_t>(nmembers));
        std::vector<int32_t> gbeg(static_cast<size_t>(nmembers));
        int64_t g = 0;
        for (int i = 0; i < nmembers; ++i) {
            // the buffer sizes gb_mesh_create and gb_solver_create allocate
            gbh::BatchMemberLayout &b = lay[size_t(i)];
            b.K = K[i];
            b.nv = nv[i];
            const int64_t groups = (K[i] + 15) / 16;
            b.etov_bytes = size_t(K[i]) * (dim + 1) * sizeof(int32_t);
            b.vstage_bytes = 5 * size_t(nv[i]) * dim * sizeof(double);
            b.wstage_bytes = 4 * size_t(nv[i]) * dim * sizeof(double);
            b.vmap_bytes = size_t(groups) * slots * 16 * sizeof(int32_t);
            b.state_bytes = size_t(groups) * 16 * NF * ref.Np * es;
            gbeg[size_t(i)] = int32_t(g);
            g += groups;
        }
        // dynamic LDS of the batched launch: the single-mesh kernel's
        // (operator fragments, slot table, staged blocks) plus the group offsets
        const size_t lds = (L.lds(ref.Nc) + 15) / 16 * 16 + size_t(nmembers) * sizeof(int32_t);
        *lds_bytes = lds;
        const std::string bad =
            gbh::check_batch_class(dim, ref.Np, NF, NFT, es, lay, gbeg, g, gbd::kMaxBatch, lds, lds_limit);
        if (!bad.empty()) return fail(GB_ERR_STATE, bad);
    } catch (const std::exception &ex) {
        return fail(GB_ERR_ARG, ex.what());
    }
    return GB_OK;
}

gb_status gb_mesh_create(gb_ctx *ctx, int dim, int N, int64_t nv, const double *vx, int64_t K, const int32_t *etov,
                         const double *period, const int8_t *face_tag, gb_mesh **out) {
    if (!ctx || !vx || !etov || !out) return fail(GB_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(GB_ERR_ARG, "dim must be 2 or 3");
    if (!supported(dim, N)) return fail(GB_ERR_UNSUPPORTED, "polynomial order not built for this dimension");
    if (nv <= 0 || K <= 0) return fail(GB_ERR_ARG, "empty mesh");
    auto m = std::make_unique<gb_mesh>();
    m->ctx = ctx;
    m->dim = dim;
    m->N = N;
    m->K = K;
    m->nv = nv;
    try {
        m->ref = gbh::build_ref_element(dim, N, 0);
    } catch (const std::exception &ex) {
        return fail(GB_ERR_ARG, ex.what());
    }
    const int nvert = dim + 1;
    // orientation: every element positively oriented
    for (int64_t e = 0; e < K; ++e) {
        double G[3][3] = {{0}};
        for (int a = 0; a < dim; ++a) {
            const int32_t v0 = etov[e * nvert], va = etov[e * nvert + a + 1];
            if (v0 < 0 || v0 >= nv || va < 0 || va >= nv) return fail(GB_ERR_ARG, "etov index out of range");
            for (int d = 0; d < dim; ++d) G[d][a] = vx[int64_t(va) * dim + d] - vx[int64_t(v0) * dim + d];
        }
        const double J = dim == 2 ? G[0][0] * G[1][1] - G[0][1] * G[1][0]
                                  : G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                                        G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                                        G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
        if (!(J > 0.0)) return fail(GB_ERR_MESH, "element " + std::to_string(e) + " is not positively oriented");
    }
    std::string err;
    m->conn = gbh::build_connectivity(m->ref, nv, vx, K, etov, period, face_tag, err);
    if (!err.empty()) return fail(GB_ERR_MESH, err);
    m->X.assign(vx, vx + nv * dim);
    GB_HIP(hipSetDevice(ctx->device));
    if (m->d_etov.alloc(size_t(K) * nvert * sizeof(int32_t)) != hipSuccess ||
        m->d_X.alloc(size_t(nv) * dim * sizeof(double)) != hipSuccess ||
        m->d_x.alloc(size_t(nv) * dim * sizeof(double)) != hipSuccess)
        return fail(GB_ERR_OOM, "device allocation for the mesh failed");
    GB_HIP(hipMemcpy(m->d_etov.p, etov, m->d_etov.bytes, hipMemcpyHostToDevice));
    GB_HIP(hipMemcpy(m->d_X.p, vx, m->d_X.bytes, hipMemcpyHostToDevice));
    GB_HIP(hipMemcpy(m->d_x.p, vx, m->d_x.bytes, hipMemcpyHostToDevice));
    {
        // blocked trace map [K/16][slots][16] (slots = face nodes rounded up to
        // a multiple of 4; -3 marks padding), checked against the flat map
        const int NFT = m->ref.Nfaces * m->ref.Nfp;
        const std::vector<int32_t> blk = gbh::blocked_trace_map(m->ref, K, m->conn);
        const std::string bad = gbh::check_mesh_tables(m->ref, nv, K, etov, m->conn, blk);
        if (!bad.empty()) return fail(GB_ERR_MESH, bad);
        if (m->d_vmapP.alloc(blk.size() * sizeof(int32_t)) != hipSuccess) return fail(GB_ERR_OOM, "vmapP");
        GB_HIP(hipMemcpy(m->d_vmapP.p, blk.data(), m->d_vmapP.bytes, hipMemcpyHostToDevice));
        // wall faces (trace map -1) for the force integral, the face node
        // lists and the integral of each face node's Lagrange function over a
        // face of measure 2: 1^T M LIFT (LIFT = M^-1 E, E the face mass)
        std::vector<int32_t> wall;
        const int Nfp = m->ref.Nfp, Nf = m->ref.Nfaces;
        for (int64_t e = 0; e < K; ++e)
            for (int f = 0; f < Nf; ++f)
                if (m->conn.vmapP[(e * Nf + f) * Nfp] == -1) wall.push_back(int32_t(e * Nf + f));
        m->nwall = int(wall.size());
        std::vector<double> wface(size_t(NFT), 0.0);
        for (int col = 0; col < NFT; ++col)
            for (int i = 0; i < m->ref.Np; ++i)
                for (int j = 0; j < m->ref.Np; ++j) wface[col] += m->ref.M(i, j) * m->ref.LIFT(j, col);
        std::vector<int32_t> fm(m->ref.fmask.begin(), m->ref.fmask.end());
        if (m->d_fmask.alloc(fm.size() * sizeof(int32_t)) != hipSuccess ||
            m->d_wface.alloc(wface.size() * sizeof(double)) != hipSuccess ||
            (!wall.empty() && m->d_wall.alloc(wall.size() * sizeof(int32_t)) != hipSuccess))
            return fail(GB_ERR_OOM, "face tables");
        GB_HIP(hipMemcpy(m->d_fmask.p, fm.data(), m->d_fmask.bytes, hipMemcpyHostToDevice));
        GB_HIP(hipMemcpy(m->d_wface.p, wface.data(), m->d_wface.bytes, hipMemcpyHostToDevice));
        if (!wall.empty()) GB_HIP(hipMemcpy(m->d_wall.p, wall.data(), m->d_wall.bytes, hipMemcpyHostToDevice));
    }
    m->motion.kind = 0;
    *out = m.release();
    return GB_OK;
}

void gb_mesh_destroy(gb_mesh *mesh) { delete mesh; }

gb_status gb_mesh_sizes(const gb_mesh *m, int64_t *K, int *Np, int *NF, int *Nfp, int *Nfaces) {
    if (!m) return fail(GB_ERR_ARG, "mesh is NULL");
    if (K) *K = m->K;
    if (Np) *Np = m->ref.Np;
    if (NF) *NF = n_fields(m->dim);
    if (Nfp) *Nfp = m->ref.Nfp;
    if (Nfaces) *Nfaces = m->ref.Nfaces;
    return GB_OK;
}

gb_status gb_mesh_vertices(const gb_mesh *m, double *vx) {
    if (!m || !vx) return fail(GB_ERR_ARG, "NULL argument");
    GB_HIP(hipSetDevice(m->ctx->device));
    GB_HIP(hipMemcpyAsync(vx, m->d_x.p, m->d_x.bytes, hipMemcpyDeviceToHost, m->ctx->stream));
    GB_HIP(hipStreamSynchronize(m->ctx->stream));
    return GB_OK;
}

gb_status gb_mesh_nodes(const gb_mesh *m, double *xyz) {
    if (!m || !xyz) return fail(GB_ERR_ARG, "NULL argument");
    std::vector<double> x(size_t(m->nv) * m->dim);
    gb_status s = gb_mesh_vertices(m, x.data());
    if (s != GB_OK) return s;
    std::vector<int32_t> etov(size_t(m->K) * (m->dim + 1));
    GB_HIP(hipMemcpy(etov.data(), m->d_etov.p, m->d_etov.bytes, hipMemcpyDeviceToHost));
    const int Np = m->ref.Np, dim = m->dim, nvert = dim + 1;
    for (int64_t e = 0; e < m->K; ++e)
        for (int d = 0; d < dim; ++d)
            for (int i = 0; i < Np; ++i) {
                double v = 0.0;
                for (int a = 0; a < nvert; ++a) v += m->ref.bary(i, a) * x[size_t(etov[e * nvert + a]) * dim + d];
                xyz[(e * dim + d) * Np + i] = v;
            }
    return GB_OK;
}

gb_status gb_set_motion(gb_mesh *m, const gb_motion *mo) {
    if (!m || !mo) return fail(GB_ERR_ARG, "NULL argument");
    if (mo->kind == GB_MOTION_VERTEX_ARRAY) return fail(GB_ERR_ARG, "vertex-array motion is set by gb_set_vertex_velocity");
    if (mo->kind < 0 || mo->kind > 5) return fail(GB_ERR_ARG, "unknown motion kind");
    if ((mo->kind == GB_MOTION_TRIPLE_PRODUCT_3D || mo->kind == GB_MOTION_FISH_3D) && m->dim != 3)
        return fail(GB_ERR_ARG, "3D motion on a 2D mesh");
    if (mo->kind == GB_MOTION_FISH_3D && !(mo->p[3] != 0.0)) return fail(GB_ERR_ARG, "fish motion needs a wavelength");
    if ((mo->kind == GB_MOTION_SIN_PRODUCT_2D || mo->kind == GB_MOTION_PLUNGE_BLEND_2D) && m->dim != 2)
        return fail(GB_ERR_ARG, "2D motion on a 3D mesh");
    m->motion.kind = mo->kind;
    for (int i = 0; i < 8; ++i) m->motion.p[i] = mo->p[i];
    m->motion.w = nullptr;
    ++m->motion_serial;
    return GB_OK;
}

gb_status gb_set_vertex_velocity(gb_mesh *m, const double *w) {
    if (!m || !w) return fail(GB_ERR_ARG, "NULL argument");
    GB_HIP(hipSetDevice(m->ctx->device));
    const size_t bytes = 4 * size_t(m->nv) * m->dim * sizeof(double);
    const bool fresh = m->motion.kind != GB_MOTION_VERTEX_ARRAY || m->d_wv.bytes != bytes;
    if (m->d_wv.bytes != bytes && m->d_wv.alloc(bytes) != hipSuccess) return fail(GB_ERR_OOM, "vertex velocities");
    // ordered after earlier work of the mesh's context that may still read it
    GB_HIP(hipStreamSynchronize(m->ctx->stream));
    GB_HIP(hipMemcpy(m->d_wv.p, w, bytes, hipMemcpyHostToDevice));
    if (fresh) {
        m->motion.kind = GB_MOTION_VERTEX_ARRAY;
        for (int i = 0; i < 8; ++i) m->motion.p[i] = 0.0;
        m->motion.w = m->d_wv.as<double>();
        ++m->motion_serial;
    }
    return GB_OK;
}

gb_status gb_solver_footprint(const gb_mesh *m, const gb_params *p, size_t *bytes) {
    if (!m || !p || !bytes) return fail(GB_ERR_ARG, "NULL argument");
    *bytes = solver_bytes(m, p);
    return GB_OK;
}

gb_status gb_mesh_footprint(const gb_mesh *m, size_t *bytes) {
    if (!m || !bytes) return fail(GB_ERR_ARG, "NULL argument");
    *bytes = mesh_bytes(m);
    return GB_OK;
}

gb_status gb_solver_create(gb_mesh *m, const gb_params *p, gb_solver **out) {
    if (!m || !p || !out) return fail(GB_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (!(p->c > 0.0) || !(p->tau > 0.0)) return fail(GB_ERR_ARG, "c and tau must be positive");
    if (p->precision != GB_FP64 && p->precision != GB_FP32) return fail(GB_ERR_ARG, "unknown precision");
    if (p->flux_mode != GB_FLUX_SPLIT && p->flux_mode != GB_FLUX_RELATIVE) return fail(GB_ERR_ARG, "unknown flux mode");
    if (m->solvers > 0)
        return fail(GB_ERR_STATE, "the mesh already has a solver (its vertex positions move with that solver)");
    auto s = std::make_unique<gb_solver>();
    s->mesh = m;
    s->prm = *p;
    s->NF = n_fields(m->dim);
    try {
        s->ref = gbh::build_ref_element(m->dim, m->N, p->cubature_degree);
    } catch (const std::exception &ex) {
        return fail(GB_ERR_ARG, ex.what());
    }
    Launcher L;
    if (!get_launcher(m->dim, m->N, p->precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel for this configuration");
    s->elem_bytes = p->precision == GB_FP32 ? 4 : 8;
    const int Np = s->ref.Np;
    const size_t need = L.lds(s->ref.Nc);
    if (need > m->ctx->max_lds) return fail(GB_ERR_UNSUPPORTED, "reference operators exceed the LDS of one workgroup");
    s->lds = need;
    s->kconst_host.assign(std::max(sizeof(gbd::KConst<double>), sizeof(gbd::KConst<float>)), 0);
    // one persistent workgroup per CU (4 or 8 wavefronts, as the kernel's
    // occupancy allows), so the operator fragments are staged in LDS once per
    // CU; measured faster than one workgroup per group, and than two
    // workgroups per CU (3D TGV 1.385 -> 1.309 ms, 2D FP64 152.5 -> 149.0 us)
    s->grid = m->ctx->num_cu;
    // Tetrahedra deal their groups round robin: the groups in flight then form
    // one contiguous window, so face neighbours a few cube rows away are
    // gathered while still in L2 (measured 3.8 % faster on the 3D TGV before
    // stage 1 read a single array; equal since); on the triangle workloads
    // both dealings measured the same.
    s->interleave = m->dim == 3;
    GB_HIP(hipSetDevice(m->ctx->device));
    const size_t n = size_t((m->K + 15) / 16 * 16) * s->NF * Np;   // padded to whole groups of 16
    if (s->Q.alloc(n * s->elem_bytes) != hipSuccess || s->A.alloc(n * s->elem_bytes) != hipSuccess ||
        s->B.alloc(n * s->elem_bytes) != hipSuccess || s->G.alloc(n * s->elem_bytes) != hipSuccess ||
        s->clock.alloc(2 * sizeof(double)) != hipSuccess || s->err.alloc(sizeof(int)) != hipSuccess ||
        s->kconst.alloc(std::max(sizeof(gbd::KConst<double>), sizeof(gbd::KConst<float>))) != hipSuccess ||
        s->vstage.alloc(5 * size_t(m->nv) * m->dim * sizeof(double)) != hipSuccess ||
        s->wstage.alloc(4 * size_t(m->nv) * m->dim * sizeof(double)) != hipSuccess)
        return fail(GB_ERR_OOM, "device allocation for the solver state failed");
    std::vector<int32_t> slots;
    if (p->precision == GB_FP64) {
        auto o = pack_ops<double>(s->ref, slots);
        if (int(o.size()) != L.ops_total(s->ref.Nc)) return fail(GB_ERR_ARG, "operator packing size mismatch");
        if (s->ops.alloc(o.size() * sizeof(double)) != hipSuccess) return fail(GB_ERR_OOM, "ops");
        GB_HIP(hipMemcpy(s->ops.p, o.data(), s->ops.bytes, hipMemcpyHostToDevice));
    } else {
        auto o = pack_ops<float>(s->ref, slots);
        if (int(o.size()) != L.ops_total(s->ref.Nc)) return fail(GB_ERR_ARG, "operator packing size mismatch");
        if (s->ops.alloc(o.size() * sizeof(float)) != hipSuccess) return fail(GB_ERR_OOM, "ops");
        GB_HIP(hipMemcpy(s->ops.p, o.data(), s->ops.bytes, hipMemcpyHostToDevice));
    }
    if (s->fmask.alloc(slots.size() * sizeof(int32_t)) != hipSuccess) return fail(GB_ERR_OOM, "slot table");
    GB_HIP(hipMemcpy(s->fmask.p, slots.data(), s->fmask.bytes, hipMemcpyHostToDevice));
    if (s->d_icub.alloc(s->ref.Icub.a.size() * sizeof(double)) != hipSuccess ||
        s->d_wcub.alloc(s->ref.cub_w.size() * sizeof(double)) != hipSuccess)
        return fail(GB_ERR_OOM, "cubature tables");
    GB_HIP(hipMemcpy(s->d_icub.p, s->ref.Icub.a.data(), s->d_icub.bytes, hipMemcpyHostToDevice));
    GB_HIP(hipMemcpy(s->d_wcub.p, s->ref.cub_w.data(), s->d_wcub.bytes, hipMemcpyHostToDevice));
    // padding elements of the last group stay zero
    for (DevBuf *b : {&s->Q, &s->A, &s->B, &s->G}) GB_HIP(hipMemset(b->p, 0, b->bytes));
    GB_HIP(hipMemset(s->err.p, 0, sizeof(int)));
    double clk[2] = {0.0, 0.0};
    GB_HIP(hipMemcpy(s->clock.p, clk, sizeof(clk), hipMemcpyHostToDevice));

    ++m->solvers;
    *out = s.release();
    return GB_OK;
}

void gb_solver_destroy(gb_solver *s) {
    if (!s) return;
    if (s->mesh) --s->mesh->solvers;
    delete s;
}

gb_status gb_state_set(gb_solver *s, const double *q, double t0) {
    if (!s || !q) return fail(GB_ERR_ARG, "NULL argument");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    gb_mesh *m = s->mesh;
    GB_HIP(hipSetDevice(m->ctx->device));
    const int64_t n = m->K * s->NF * s->ref.Np;
    DevBuf tmp;
    if (tmp.alloc(size_t(n) * sizeof(double)) != hipSuccess) return fail(GB_ERR_OOM, "staging buffer");
    hipStream_t st = m->ctx->stream;
    GB_HIP(hipMemcpyAsync(tmp.p, q, size_t(n) * sizeof(double), hipMemcpyHostToDevice, st));
    const unsigned nb = unsigned((n + 255) / 256);
    const double rho0 = s->prm.precision == GB_FP32 ? s->prm.rho0 : 0.0;
    if (s->prm.precision == GB_FP64)
        hipLaunchKernelGGL(to_state_kernel<double>, dim3(nb), dim3(256), 0, st, tmp.as<double>(), s->Q.as<double>(), n,
                           s->ref.Np, s->NF, 0.0);
    else
        hipLaunchKernelGGL(to_state_kernel<float>, dim3(nb), dim3(256), 0, st, tmp.as<double>(), s->Q.as<float>(), n,
                           s->ref.Np, s->NF, rho0);
    GB_HIP(hipGetLastError());
    return reset_clock_and_positions(s, t0);
}

gb_status gb_state_set_equilibrium(gb_solver *s, const double *rho, const double *u, const double *offset,
                                   double t0) {
    if (!s || !rho || !u) return fail(GB_ERR_ARG, "NULL argument");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    gb_mesh *m = s->mesh;
    GB_HIP(hipSetDevice(m->ctx->device));
    const int64_t n = m->K * s->ref.Np;
    const int dim = m->dim;
    DevBuf tmp, bad;
    if (tmp.alloc(size_t(n) * (1 + dim) * sizeof(double) + 10 * sizeof(double)) != hipSuccess ||
        bad.alloc(sizeof(int)) != hipSuccess)
        return fail(GB_ERR_OOM, "staging buffer");
    hipStream_t st = m->ctx->stream;
    double *d_rho = tmp.as<double>(), *d_u = d_rho + n, *d_off = d_u + n * dim;
    GB_HIP(hipMemcpyAsync(d_rho, rho, size_t(n) * sizeof(double), hipMemcpyHostToDevice, st));
    GB_HIP(hipMemcpyAsync(d_u, u, size_t(n) * dim * sizeof(double), hipMemcpyHostToDevice, st));
    if (offset) GB_HIP(hipMemcpyAsync(d_off, offset, size_t(s->NF) * sizeof(double), hipMemcpyHostToDevice, st));
    GB_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
    const unsigned nb = unsigned((n + 255) / 256);
    const double rho0 = s->prm.precision == GB_FP32 ? s->prm.rho0 : 0.0;
    const double *po = offset ? d_off : nullptr;
    int *pb = bad.as<int>();
    if (dim == 2 && s->prm.precision == GB_FP64)
        hipLaunchKernelGGL((gbd::equilibrium_kernel<2, double>), dim3(nb), dim3(256), 0, st, d_rho, d_u, po, m->K,
                           s->ref.Np, s->prm.c, 0.0, s->Q.as<double>(), pb);
    else if (dim == 2)
        hipLaunchKernelGGL((gbd::equilibrium_kernel<2, float>), dim3(nb), dim3(256), 0, st, d_rho, d_u, po, m->K,
                           s->ref.Np, s->prm.c, rho0, s->Q.as<float>(), pb);
    else if (s->prm.precision == GB_FP64)
        hipLaunchKernelGGL((gbd::equilibrium_kernel<3, double>), dim3(nb), dim3(256), 0, st, d_rho, d_u, po, m->K,
                           s->ref.Np, s->prm.c, 0.0, s->Q.as<double>(), pb);
    else
        hipLaunchKernelGGL((gbd::equilibrium_kernel<3, float>), dim3(nb), dim3(256), 0, st, d_rho, d_u, po, m->K,
                           s->ref.Np, s->prm.c, rho0, s->Q.as<float>(), pb);
    GB_HIP(hipGetLastError());
    int flag = 0;
    GB_HIP(hipMemcpyAsync(&flag, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    if (flag) {
        s->has_state = false;
        return fail(GB_ERR_ARG, "a density is not positive");
    }
    return reset_clock_and_positions(s, t0);
}

gb_status gb_equilibrium_moments(int dim, double c, int64_t n, const double *rho, const double *u, double *q) {
    if (!rho || !u || !q) return fail(GB_ERR_ARG, "NULL argument");
    if (dim != 2 && dim != 3) return fail(GB_ERR_ARG, "dim must be 2 or 3");
    if (!(c > 0.0) || n < 0) return fail(GB_ERR_ARG, "c must be positive and n >= 0");
    const double s2 = std::sqrt(2.0);
    for (int64_t i = 0; i < n; ++i) {
        const double r = rho[i];
        if (!(r > 0.0)) return fail(GB_ERR_ARG, "a density is not positive");
        double m[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) m[d] = r * u[d * n + i] / c;
        q[0 * n + i] = r;
        for (int d = 0; d < dim; ++d) q[(1 + d) * n + i] = m[d];
        if (dim == 2) {
            q[3 * n + i] = m[0] * m[1] / r;
            q[4 * n + i] = m[0] * m[0] / (s2 * r);
            q[5 * n + i] = m[1] * m[1] / (s2 * r);
        } else {
            q[4 * n + i] = m[0] * m[1] / r;
            q[5 * n + i] = m[0] * m[2] / r;
            q[6 * n + i] = m[1] * m[2] / r;
            q[7 * n + i] = m[0] * m[0] / (s2 * r);
            q[8 * n + i] = m[1] * m[1] / (s2 * r);
            q[9 * n + i] = m[2] * m[2] / (s2 * r);
        }
    }
    return GB_OK;
}

}  // extern "C"

namespace {
struct CheckpointHeader {
    char magic[8];
    int32_t dim, N, precision, NF;
    int64_t K, nv, state_bytes, vertex_bytes;
    double clock[2];
};
constexpr char kCheckpointMagic[8] = {'g', 'b', 'c', 'k', 'p', 't', '0', '1'};

size_t state_storage_bytes(const gb_solver *s) {
    return size_t((s->mesh->K + 15) / 16 * 16) * s->NF * s->ref.Np * s->elem_bytes;
}
}  // namespace

extern "C" {

gb_status gb_checkpoint_bytes(const gb_solver *s, size_t *bytes) {
    if (!s || !bytes) return fail(GB_ERR_ARG, "NULL argument");
    *bytes = sizeof(CheckpointHeader) + state_storage_bytes(s) + s->mesh->d_x.bytes;
    return GB_OK;
}

gb_status gb_checkpoint_save(gb_solver *s, void *buf, size_t bytes) {
    if (!s || !buf) return fail(GB_ERR_ARG, "NULL argument");
    if (!s->has_state) return fail(GB_ERR_STATE, "no state set");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    size_t need = 0;
    gb_checkpoint_bytes(s, &need);
    if (bytes < need) return fail(GB_ERR_ARG, "checkpoint buffer too small");
    gb_mesh *m = s->mesh;
    GB_HIP(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    CheckpointHeader h{};
    std::memcpy(h.magic, kCheckpointMagic, 8);
    h.dim = m->dim;
    h.N = m->N;
    h.precision = s->prm.precision;
    h.NF = s->NF;
    h.K = m->K;
    h.nv = m->nv;
    h.state_bytes = int64_t(state_storage_bytes(s));
    h.vertex_bytes = int64_t(m->d_x.bytes);
    unsigned char *out = static_cast<unsigned char *>(buf);
    GB_HIP(hipMemcpyAsync(h.clock, s->clock.p, sizeof(h.clock), hipMemcpyDeviceToHost, st));
    GB_HIP(hipMemcpyAsync(out + sizeof(h), s->Q.p, size_t(h.state_bytes), hipMemcpyDeviceToHost, st));
    GB_HIP(hipMemcpyAsync(out + sizeof(h) + h.state_bytes, m->d_x.p, size_t(h.vertex_bytes), hipMemcpyDeviceToHost,
                          st));
    GB_HIP(hipStreamSynchronize(st));
    std::memcpy(out, &h, sizeof(h));
    return check_error_flag(s);
}

gb_status gb_checkpoint_load(gb_solver *s, const void *buf, size_t bytes) {
    if (!s || !buf) return fail(GB_ERR_ARG, "NULL argument");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    gb_mesh *m = s->mesh;
    CheckpointHeader h;
    if (bytes < sizeof(h)) return fail(GB_ERR_ARG, "checkpoint buffer too small");
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, kCheckpointMagic, 8) != 0) return fail(GB_ERR_ARG, "not a checkpoint");
    if (h.dim != m->dim || h.N != m->N || h.precision != s->prm.precision || h.NF != s->NF || h.K != m->K ||
        h.nv != m->nv || h.state_bytes != int64_t(state_storage_bytes(s)) || h.vertex_bytes != int64_t(m->d_x.bytes))
        return fail(GB_ERR_ARG, "checkpoint of another mesh, order or precision");
    if (bytes < sizeof(h) + size_t(h.state_bytes + h.vertex_bytes)) return fail(GB_ERR_ARG, "checkpoint truncated");
    GB_HIP(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    const unsigned char *in = static_cast<const unsigned char *>(buf);
    GB_HIP(hipMemcpyAsync(s->Q.p, in + sizeof(h), size_t(h.state_bytes), hipMemcpyHostToDevice, st));
    GB_HIP(hipMemcpyAsync(m->d_x.p, in + sizeof(h) + h.state_bytes, size_t(h.vertex_bytes), hipMemcpyHostToDevice,
                          st));
    GB_HIP(hipMemcpyAsync(s->clock.p, h.clock, sizeof(h.clock), hipMemcpyHostToDevice, st));
    GB_HIP(hipMemsetAsync(s->err.p, 0, sizeof(int), st));
    GB_HIP(hipStreamSynchronize(st));
    s->t = h.clock[0];
    s->step = int64_t(h.clock[1]);
    s->has_state = true;
    return GB_OK;
}

gb_status gb_state_get(gb_solver *s, double *q, double *t, int64_t *step) {
    if (!s) return fail(GB_ERR_ARG, "NULL solver");
    if (!s->has_state) return fail(GB_ERR_STATE, "no state set");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    gb_mesh *m = s->mesh;
    GB_HIP(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    gb_status es = check_error_flag(s);
    if (q) {
        const int64_t n = m->K * s->NF * s->ref.Np;
        DevBuf tmp;
        if (tmp.alloc(size_t(n) * sizeof(double)) != hipSuccess) return fail(GB_ERR_OOM, "staging buffer");
        const unsigned nb = unsigned((n + 255) / 256);
        if (s->prm.precision == GB_FP64)
            hipLaunchKernelGGL(from_state_kernel<double>, dim3(nb), dim3(256), 0, st, s->Q.as<double>(),
                               tmp.as<double>(), n, s->ref.Np, s->NF, 0.0);
        else
            hipLaunchKernelGGL(from_state_kernel<float>, dim3(nb), dim3(256), 0, st, s->Q.as<float>(),
                               tmp.as<double>(), n, s->ref.Np, s->NF, s->prm.rho0);
        GB_HIP(hipGetLastError());
        GB_HIP(hipMemcpyAsync(q, tmp.p, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    double clk[2];
    GB_HIP(hipMemcpyAsync(clk, s->clock.p, sizeof(clk), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    if (t) *t = clk[0];
    if (step) *step = int64_t(clk[1]);
    return es;
}

gb_status gb_rhs(gb_solver *s, const double *q, double *F) {
    if (!s || !q || !F) return fail(GB_ERR_ARG, "NULL argument");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    gb_mesh *m = s->mesh;
    Launcher L;
    if (!get_launcher(m->dim, m->N, s->prm.precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel");
    GB_HIP(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    const int64_t n = m->K * s->NF * s->ref.Np;
    const int64_t npad = (m->K + 15) / 16 * 16 * s->NF * s->ref.Np;
    DevBuf dq, din, dout;
    if (dq.alloc(size_t(n) * sizeof(double)) != hipSuccess || din.alloc(size_t(npad) * s->elem_bytes) != hipSuccess ||
        dout.alloc(size_t(npad) * s->elem_bytes) != hipSuccess)
        return fail(GB_ERR_OOM, "rhs buffers");
    GB_HIP(hipMemsetAsync(din.p, 0, din.bytes, st));
    GB_HIP(hipMemcpyAsync(dq.p, q, size_t(n) * sizeof(double), hipMemcpyHostToDevice, st));
    const unsigned nb = unsigned((n + 255) / 256);
    const double rho0 = s->prm.precision == GB_FP32 ? s->prm.rho0 : 0.0;
    if (s->prm.precision == GB_FP64)
        hipLaunchKernelGGL(to_state_kernel<double>, dim3(nb), dim3(256), 0, st, dq.as<double>(), din.as<double>(), n,
                           s->ref.Np, s->NF, 0.0);
    else
        hipLaunchKernelGGL(to_state_kernel<float>, dim3(nb), dim3(256), 0, st, dq.as<double>(), din.as<float>(), n,
                           s->ref.Np, s->NF, rho0);
    GB_HIP(hipGetLastError());
    {
        hipError_t pe = ensure_consts(s, L, st);
        if (pe != hipSuccess) return fail(GB_ERR_DEVICE, std::string("constants upload: ") + hipGetErrorString(pe));
    }
    {
        hipError_t me = launch_motion(s, 0.0, st);
        if (me != hipSuccess) return fail(GB_ERR_DEVICE, std::string("motion: ") + hipGetErrorString(me));
    }
    // point the state slots at the scratch buffers for one RHS-only launch
    std::swap(s->Q.p, din.p);
    std::swap(s->A.p, dout.p);
    hipError_t le = L.stage(s, 4, 0.0, st);
    std::swap(s->Q.p, din.p);
    std::swap(s->A.p, dout.p);
    if (le != hipSuccess) return fail(GB_ERR_DEVICE, std::string("rhs launch: ") + hipGetErrorString(le));
    if (s->prm.precision == GB_FP64)
        hipLaunchKernelGGL(from_state_kernel<double>, dim3(nb), dim3(256), 0, st, dout.as<double>(), dq.as<double>(), n,
                           s->ref.Np, s->NF, 0.0);
    else
        hipLaunchKernelGGL(from_state_kernel<float>, dim3(nb), dim3(256), 0, st, dout.as<float>(), dq.as<double>(), n,
                           s->ref.Np, s->NF, 0.0);
    GB_HIP(hipGetLastError());
    GB_HIP(hipMemcpyAsync(F, dq.p, size_t(n) * sizeof(double), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    return check_error_flag(s);
}

}  // extern "C"

namespace {

// Workgroups of the energy reduction: one wavefront per element, at most a
// few workgroups per CU (the per-element work is small).
int energy_grid(const gb_solver *s) {
    const int64_t waves = s->mesh->K;
    const int64_t per_block = gbd::kDiagBlock / 64;
    return int(std::max<int64_t>(1, std::min<int64_t>(int64_t(s->mesh->ctx->num_cu) * 4,
                                                      (waves + per_block - 1) / per_block)));
}

// The register form of the energy kernel serves rules of up to 128 points
// on the built orders (its node count is a template parameter).
bool energy_in_registers(const gb_solver *s) {
    const int Np = s->ref.Np;
    const bool np_ok = s->mesh->dim == 2 ? (Np == 3 || Np == 6 || Np == 10 || Np == 15 || Np == 21)
                                         : (Np == 4 || Np == 10 || Np == 20);
    return s->ref.Nc <= 128 && np_ok;
}

size_t energy_lds(const gb_solver *s) {
    const int NC = s->mesh->dim + 1, Np = s->ref.Np, Nc = s->ref.Nc;
    const size_t waves = gbd::kDiagBlock / 64;
    if (energy_in_registers(s)) return sizeof(double) * (gbd::kDiagBlock + waves * 2 * NC * Np);
    return sizeof(double) * (size_t(Nc) * Np + Nc + gbd::kDiagBlock + waves * 2 * NC * Np);
}

// Enqueue the energy diagnostic: the current geometry and grid velocity
// (vertex kernel with dt = 0), F(q) into the free array A, the per-workgroup
// partial sums into partial[grid][4] and {E_K, -dE_K/dt, |Omega|} into
// result[3].  Needs the solver's constants on the device.
gb_status enqueue_energy(gb_solver *s, const Launcher &L, double rho_inf, double *partial, double *result,
                         hipStream_t st) {
    gb_mesh *m = s->mesh;
    GB_HIP(launch_motion(s, 0.0, st));
    GB_HIP(L.stage(s, 4, 0.0, st));
    const int grid = energy_grid(s);
    const size_t lds = energy_lds(s);
    const double rho0 = s->prm.precision == GB_FP32 ? s->prm.rho0 : 0.0;
    auto run = [&](auto tag, auto dimc) -> hipError_t {
        using T = decltype(tag);
        constexpr int D = decltype(dimc)::value;
        gbd::EnergyArgs<T> a{};
        a.K = m->K;
        a.Np = s->ref.Np;
        a.NF = s->NF;
        a.Nc = s->ref.Nc;
        a.dim = D;
        a.Q = s->Q.as<T>();
        a.F = s->A.as<T>();
        a.etov = m->d_etov.as<int32_t>();
        a.x = s->vstage.as<double>();   // slot 0: the current positions
        a.w = s->wstage.as<double>();   // slot 0: the grid velocity at the current time
        a.Icub = s->d_icub.as<double>();
        a.wcub = s->d_wcub.as<double>();
        a.c = s->prm.c;
        a.rho0 = rho0;
        a.partial = partial;
        auto reg = [&](auto npc) {
            constexpr int NP = decltype(npc)::value;
            hipLaunchKernelGGL((gbd::energy_partial_reg_kernel<D, T, NP>), dim3(grid), dim3(gbd::kDiagBlock), lds, st, a);
        };
        if (energy_in_registers(s)) {
            if constexpr (D == 2) {
                switch (a.Np) {
                    case 3: reg(std::integral_constant<int, 3>{}); break;
                    case 6: reg(std::integral_constant<int, 6>{}); break;
                    case 10: reg(std::integral_constant<int, 10>{}); break;
                    case 15: reg(std::integral_constant<int, 15>{}); break;
                    default: reg(std::integral_constant<int, 21>{}); break;
                }
            } else {
                switch (a.Np) {
                    case 4: reg(std::integral_constant<int, 4>{}); break;
                    case 10: reg(std::integral_constant<int, 10>{}); break;
                    default: reg(std::integral_constant<int, 20>{}); break;
                }
            }
        } else hipLaunchKernelGGL((gbd::energy_partial_kernel<D, T>), dim3(grid), dim3(gbd::kDiagBlock), lds, st, a);
        return hipGetLastError();
    };
    hipError_t e;
    if (m->dim == 2)
        e = s->prm.precision == GB_FP64 ? run(double{}, std::integral_constant<int, 2>{})
                                        : run(float{}, std::integral_constant<int, 2>{});
    else
        e = s->prm.precision == GB_FP64 ? run(double{}, std::integral_constant<int, 3>{})
                                        : run(float{}, std::integral_constant<int, 3>{});
    GB_HIP(e);
    hipLaunchKernelGGL(gbd::energy_final_kernel, dim3(1), dim3(gbd::kDiagBlock), 0, st, partial, grid, rho_inf,
                       result);
    GB_HIP(hipGetLastError());
    return GB_OK;
}

gb_status check_diag_call(gb_solver *s, Launcher &L) {
    if (!s->has_state) return fail(GB_ERR_STATE, "no state set");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    gb_mesh *m = s->mesh;
    if (!get_launcher(m->dim, m->N, s->prm.precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel");
    GB_HIP(hipSetDevice(m->ctx->device));
    GB_HIP(ensure_consts(s, L, m->ctx->stream));
    return GB_OK;
}

}  // namespace

extern "C" {

gb_status gb_energy(gb_solver *s, double rho_inf, double out[3]) {
    if (!s || !out) return fail(GB_ERR_ARG, "NULL argument");
    if (!(rho_inf > 0.0)) return fail(GB_ERR_ARG, "rho_inf must be positive");
    Launcher L;
    gb_status r = check_diag_call(s, L);
    if (r != GB_OK) return r;
    const int grid = energy_grid(s);
    const size_t need = (size_t(grid) * gbd::kDiagSums + 4) * sizeof(double);
    if (s->diag.bytes < need && s->diag.alloc(need) != hipSuccess) return fail(GB_ERR_OOM, "energy reduction buffer");
    hipStream_t st = s->mesh->ctx->stream;
    double *partial = s->diag.as<double>();
    double *result = partial + size_t(grid) * gbd::kDiagSums;
    r = enqueue_energy(s, L, rho_inf, partial, result, st);
    if (r != GB_OK) return r;
    GB_HIP(hipMemcpyAsync(out, result, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    return check_error_flag(s);
}

gb_status gb_energy_noalloc(gb_solver *s, double rho_inf, double out[3]) {
    if (!s || !out) return fail(GB_ERR_ARG, "NULL argument");
    if (!(rho_inf > 0.0)) return fail(GB_ERR_ARG, "rho_inf must be positive");
    Launcher L;
    gb_status r = check_diag_call(s, L);
    if (r != GB_OK) return r;
    const int grid = energy_grid(s);
    const size_t need = size_t(grid) * gbd::kDiagSums + 4;
    if (need > kScratchDoubles)
        return fail(GB_ERR_ARG, "the reduction needs " + std::to_string(need) + " doubles of scratch, more than the " +
                                    std::to_string(kScratchDoubles) + " of the allocation-free form");
    gb_ctx *ctx = s->mesh->ctx;
    if (!ctx->scratch) return fail(GB_ERR_STATE, "no scratch address for this device");
    hipStream_t st = ctx->stream;
    // every workgroup writes all of its partial sums and the final pass
    // writes the whole result, so nothing has to be cleared first
    double *partial = ctx->scratch;
    double *result = partial + size_t(grid) * gbd::kDiagSums;
    r = enqueue_energy(s, L, rho_inf, partial, result, st);
    if (r != GB_OK) return r;
    GB_HIP(hipMemcpyAsync(out, result, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    return check_error_flag(s);
}

gb_status gb_wall_force(gb_solver *s, double *out) {
    if (!s || !out) return fail(GB_ERR_ARG, "NULL argument");
    Launcher L;
    gb_status r = check_diag_call(s, L);
    if (r != GB_OK) return r;
    gb_mesh *m = s->mesh;
    const int dim = m->dim;
    for (int k = 0; k < 2 * dim; ++k) out[k] = 0.0;
    if (m->nwall == 0) return GB_OK;
    const size_t need = 8 * sizeof(double);
    if (s->diag.bytes < need && s->diag.alloc(need) != hipSuccess) return fail(GB_ERR_OOM, "force reduction buffer");
    hipStream_t st = m->ctx->stream;
    const double rho0 = s->prm.precision == GB_FP32 ? s->prm.rho0 : 0.0;
    auto run = [&](auto tag, auto dimc) -> hipError_t {
        using T = decltype(tag);
        constexpr int D = decltype(dimc)::value;
        gbd::ForceArgs<T> a{};
        a.nwall = m->nwall;
        a.wall = m->d_wall.as<int32_t>();
        a.Np = s->ref.Np;
        a.NF = s->NF;
        a.Nfp = s->ref.Nfp;
        a.Q = s->Q.as<T>();
        a.etov = m->d_etov.as<int32_t>();
        a.x = m->d_x.as<double>();
        a.fmask = m->d_fmask.as<int32_t>();
        a.wface = m->d_wface.as<double>();
        a.c = s->prm.c;
        a.rho0 = rho0;
        a.out = s->diag.as<double>();
        hipLaunchKernelGGL((gbd::wall_force_kernel<D, T>), dim3(1), dim3(gbd::kDiagBlock), 0, st, a);
        return hipGetLastError();
    };
    hipError_t e;
    if (dim == 2)
        e = s->prm.precision == GB_FP64 ? run(double{}, std::integral_constant<int, 2>{})
                                        : run(float{}, std::integral_constant<int, 2>{});
    else
        e = s->prm.precision == GB_FP64 ? run(double{}, std::integral_constant<int, 3>{})
                                        : run(float{}, std::integral_constant<int, 3>{});
    GB_HIP(e);
    GB_HIP(hipMemcpyAsync(out, s->diag.p, 2 * dim * sizeof(double), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    return check_error_flag(s);
}

gb_status gb_sark_step(gb_solver *s, double dt, int64_t nsteps) {
    if (!s) return fail(GB_ERR_ARG, "NULL solver");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    if (!s->has_state) return fail(GB_ERR_STATE, "no state set");
    if (!(dt > 0.0) || nsteps < 0) return fail(GB_ERR_ARG, "dt must be positive and nsteps >= 0");
    gb_mesh *m = s->mesh;
    Launcher L;
    if (!get_launcher(m->dim, m->N, s->prm.precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel");
    GB_HIP(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    GB_HIP(L.prepare(s, dt, st));
    for (int64_t k = 0; k < nsteps; ++k) {
        gb_status r = enqueue_step(s, L, dt, st);
        if (r != GB_OK) return r;
    }
    s->step += nsteps;
    return GB_OK;
}

gb_status gb_sark_step_graph(gb_solver *s, double dt, int64_t nsteps) {
    if (!s) return fail(GB_ERR_ARG, "NULL solver");
    if (s->in_batch) return fail(GB_ERR_STATE, "the solver is a member of a batch");
    if (!s->has_state) return fail(GB_ERR_STATE, "no state set");
    if (!(dt > 0.0) || nsteps < 0) return fail(GB_ERR_ARG, "dt must be positive and nsteps >= 0");
    gb_mesh *m = s->mesh;
    Launcher L;
    if (!get_launcher(m->dim, m->N, s->prm.precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel");
    GB_HIP(hipSetDevice(m->ctx->device));
    hipStream_t st = m->ctx->stream;
    GB_HIP(L.prepare(s, dt, st));
    if (!s->graph_exec || s->graph_dt != dt || s->graph_motion_serial != m->motion_serial) {
        if (s->graph_exec) {
            GB_HIP(hipGraphExecDestroy(s->graph_exec));
            s->graph_exec = nullptr;
        }
        // capture on a private stream (the legacy default stream cannot be captured)
        hipStream_t cap;
        GB_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        const bool timing = s->timing;
        s->timing = false;
        hipGraph_t g;
        GB_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        gb_status r = enqueue_step(s, L, dt, cap);
        hipError_t ce = hipStreamEndCapture(cap, &g);
        s->timing = timing;
        (void)hipStreamDestroy(cap);
        if (r != GB_OK) return r;
        if (ce != hipSuccess) return fail(GB_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(GB_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
        s->graph_dt = dt;
        s->graph_motion_serial = m->motion_serial;
    }
    for (int64_t k = 0; k < nsteps; ++k) GB_HIP(hipGraphLaunch(s->graph_exec, st));
    s->step += nsteps;
    return GB_OK;
}

static gb_status resolve_events(gb_solver *s) {
    if (s->ev.empty()) return GB_OK;
    GB_HIP(hipEventSynchronize(s->ev.back()));
    for (size_t p = 0; p + 1 < s->ev.size(); p += 2) {
        float ms = 0.f;
        GB_HIP(hipEventElapsedTime(&ms, s->ev[p], s->ev[p + 1]));
        const int kind = s->ev_kind[p / 2];
        s->time_ms += ms;
        s->time_ms_kind[kind] += ms;
        ++s->time_launches;
        ++s->launches_kind[kind];
    }
    for (auto e : s->ev) (void)hipEventDestroy(e);
    s->ev.clear();
    s->ev_kind.clear();
    return GB_OK;
}

gb_status gb_solver_time_stages(gb_solver *s, int enable) {
    if (!s) return fail(GB_ERR_ARG, "NULL solver");
    gb_status r = resolve_events(s);
    if (r != GB_OK) return r;
    s->timing = enable != 0;
    s->time_ms = 0.0;
    s->time_launches = 0;
    for (int k = 0; k < 4; ++k) {
        s->time_ms_kind[k] = 0.0;
        s->launches_kind[k] = 0;
    }
    return GB_OK;
}

gb_status gb_solver_stage_time(gb_solver *s, double *avg_ms, int64_t *launches) {
    if (!s) return fail(GB_ERR_ARG, "NULL solver");
    gb_status r = resolve_events(s);
    if (r != GB_OK) return r;
    if (avg_ms) *avg_ms = s->time_launches ? s->time_ms / double(s->time_launches) : 0.0;
    if (launches) *launches = s->time_launches;
    return GB_OK;
}

gb_status gb_solver_stage_time_by_kind(gb_solver *s, double *avg_ms4) {
    if (!s || !avg_ms4) return fail(GB_ERR_ARG, "NULL argument");
    gb_status r = resolve_events(s);
    if (r != GB_OK) return r;
    for (int k = 0; k < 4; ++k) avg_ms4[k] = s->launches_kind[k] ? s->time_ms_kind[k] / double(s->launches_kind[k]) : 0.0;
    return GB_OK;
}

gb_status gb_batch_create(gb_ctx *ctx, size_t hbm_budget, gb_batch **out) {
    if (!ctx || !out) return fail(GB_ERR_ARG, "NULL argument");
    auto b = std::make_unique<gb_batch>();
    b->ctx = ctx;
    b->budget = hbm_budget;
    *out = b.release();
    return GB_OK;
}

void gb_batch_destroy(gb_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    for (auto &mb : b->members) mb.s->in_batch = false;
    delete b;
}

gb_status gb_batch_add(gb_batch *b, gb_solver *s, double dt, int64_t nsteps, uint64_t *ticket) {
    if (!b || !s || !ticket) return fail(GB_ERR_ARG, "NULL argument");
    if (!s->has_state) return fail(GB_ERR_STATE, "no state set");
    if (!(dt > 0.0) || nsteps < 1) return fail(GB_ERR_ARG, "dt must be positive and nsteps >= 1");
    gb_mesh *m = s->mesh;
    if (m->ctx->device != b->ctx->device) return fail(GB_ERR_ARG, "solver lives on another device");
    for (const auto &mb : b->members)
        if (mb.s == s) return fail(GB_ERR_STATE, "solver is already in the batch");
    if (int(b->members.size()) >= gbd::kMaxBatch) return fail(GB_ERR_BUSY, "batch is full");
    const size_t bytes = solver_bytes(m, &s->prm) + mesh_bytes(m);
    if (b->used + bytes > b->budget) return fail(GB_ERR_BUSY, "request does not fit the free budget of the batch");
    Launcher L;
    if (!get_launcher(m->dim, m->N, s->prm.precision, L)) return fail(GB_ERR_UNSUPPORTED, "no kernel");
    if (!L.shape.batch_stage)
        return fail(GB_ERR_UNSUPPORTED, "the batched form is not built for this element shape and precision");
    GB_HIP(hipSetDevice(m->ctx->device));
    {
        size_t scratch = 0;
        GB_HIP(L.shape.batch_scratch(&scratch));
        if (scratch) return fail(GB_ERR_UNSUPPORTED, "the batched kernel of this shape needs scratch memory");
    }
    GB_HIP(L.prepare(s, dt, m->ctx->stream));
    double clk[2];
    GB_HIP(hipMemcpyAsync(clk, s->clock.p, sizeof(clk), hipMemcpyDeviceToHost, m->ctx->stream));
    GB_HIP(hipStreamSynchronize(m->ctx->stream));
    gb_batch::Member mb;
    mb.s = s;
    mb.dt = dt;
    mb.target = clk[1] + double(nsteps);
    mb.ticket = b->next_ticket++;
    mb.bytes = bytes;
    s->in_batch = true;
    b->members.push_back(mb);
    b->used += bytes;
    b->dirty = true;
    *ticket = mb.ticket;
    return GB_OK;
}

gb_status gb_batch_run(gb_batch *b, int64_t steps) {
    if (!b) return fail(GB_ERR_ARG, "NULL batch");
    if (steps < 0) return fail(GB_ERR_ARG, "steps must be >= 0");
    if (b->dirty) {
        const gb_status r = batch_rebuild(b);
        if (r != GB_OK) return r;
    }
    if (b->members.empty() || steps == 0) return GB_OK;
    // the graph holds k steps, k the largest divisor of `steps` up to 8
    int k = 1;
    for (int d = 8; d >= 1; --d)
        if (steps % d == 0) {
            k = d;
            break;
        }
    GB_HIP(hipSetDevice(b->ctx->device));
    const bool small = has_small(b);
    if (small && (!b->graph || b->graph_steps != k)) {
        GB_HIP(hipStreamSynchronize(b->ctx->stream));
        const gb_status r = batch_capture(b, k);
        if (r != GB_OK) return r;
    }
    {
        const gb_status r = ensure_aux(b);
        if (r != GB_OK) return r;
    }
    // as many auxiliary streams as there are solo members, at most the
    // concurrency; they start after the work already on the batch's stream
    const int use = b->concurrency > 1 ? std::min(int(b->aux.size()), solo_count(b)) : 0;
    if (use > 1) {
        GB_HIP(hipEventRecord(b->fork_ev, b->ctx->stream));
        for (int i = 0; i < use; ++i) GB_HIP(hipStreamWaitEvent(b->aux[size_t(i)], b->fork_ev, 0));
    }
    hipError_t le = hipSuccess;
    for (int64_t n = 0; n < steps / k && le == hipSuccess; ++n) {
        le = batch_launch_solo(b, k, b->ctx->stream, use);
        if (small && le == hipSuccess) le = hipGraphLaunch(b->graph, b->ctx->stream);
    }
    // the batch's stream waits for the auxiliary streams, so a synchronisation
    // of it (gb_batch_poll, the next table rebuild) covers every member
    for (int i = 0; use > 1 && i < use; ++i) {
        const hipError_t e = hipEventRecord(b->join_ev[size_t(i)], b->aux[size_t(i)]);
        if (e == hipSuccess) GB_HIP(hipStreamWaitEvent(b->ctx->stream, b->join_ev[size_t(i)], 0));
        else if (le == hipSuccess) le = e;
    }
    GB_HIP(le);
    return GB_OK;
}

gb_status gb_batch_poll(gb_batch *b, uint64_t *done, int capacity, int *n_done) {
    if (!b || !n_done || (capacity > 0 && !done)) return fail(GB_ERR_ARG, "NULL argument");
    *n_done = 0;
    GB_HIP(hipSetDevice(b->ctx->device));
    hipStream_t st = b->ctx->stream;
    std::vector<double> clk(2 * b->members.size());
    for (size_t i = 0; i < b->members.size(); ++i)
        GB_HIP(hipMemcpyAsync(&clk[2 * i], b->members[i].s->clock.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    GB_HIP(hipStreamSynchronize(st));
    std::vector<gb_batch::Member> keep;
    for (size_t i = 0; i < b->members.size(); ++i) {
        gb_batch::Member &mb = b->members[i];
        if (clk[2 * i + 1] >= mb.target && *n_done < capacity) {
            done[(*n_done)++] = mb.ticket;
            mb.s->t = clk[2 * i];
            mb.s->step = int64_t(clk[2 * i + 1]);
            mb.s->in_batch = false;
            b->used -= mb.bytes;
            b->dirty = true;
        } else {
            keep.push_back(mb);
        }
    }
    b->members.swap(keep);
    return GB_OK;
}

gb_status gb_batch_info(const gb_batch *b, int *active, size_t *used_bytes, size_t *budget) {
    if (!b) return fail(GB_ERR_ARG, "NULL batch");
    if (active) *active = int(b->members.size());
    if (used_bytes) *used_bytes = b->used;
    if (budget) *budget = b->budget;
    return GB_OK;
}

gb_status gb_batch_set_concurrency(gb_batch *b, int streams) {
    if (!b) return fail(GB_ERR_ARG, "NULL batch");
    if (streams < 1 || streams > 8) return fail(GB_ERR_ARG, "streams must be 1..8");
    GB_HIP(hipSetDevice(b->ctx->device));
    GB_HIP(hipStreamSynchronize(b->ctx->stream));
    b->concurrency = streams;
    return GB_OK;
}

gb_status gb_batch_set_autotune(gb_batch *b, int enable) {
    if (!b) return fail(GB_ERR_ARG, "NULL batch");
    b->autotune = enable != 0;
    return GB_OK;
}

gb_status gb_batch_class_count(const gb_batch *b, int *n) {
    if (!b || !n) return fail(GB_ERR_ARG, "NULL argument");
    *n = int(b->classes.size());
    return GB_OK;
}

gb_status gb_batch_class_tile(const gb_batch *b, int i, int64_t *tile) {
    if (!b || !tile) return fail(GB_ERR_ARG, "NULL argument");
    if (i < 0 || i >= int(b->classes.size())) return fail(GB_ERR_ARG, "class index out of range");
    const gb_batch::Class &c = b->classes[size_t(i)];
    tile[0] = c.grid;
    tile[1] = c.waves;
    tile[2] = c.interleave ? 1 : 0;
    return GB_OK;
}

gb_status gb_tune_cache_save(const char *path) {
    if (!path) return fail(GB_ERR_ARG, "NULL path");
    std::lock_guard<std::mutex> lk(g_tile_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(GB_ERR_ARG, std::string("cannot write ") + path);
    std::fprintf(f, "# gb launch tiles: arch dim N precision Nc solo group-bucket : grid waves interleave\n");
    for (const auto &kv : g_tiles)
        std::fprintf(f, "%s : %d %d %d\n", kv.first.c_str(), kv.second.grid, kv.second.waves, kv.second.interleave);
    std::fclose(f);
    return GB_OK;
}

gb_status gb_tune_cache_load(const char *path, int *entries) {
    if (!path) return fail(GB_ERR_ARG, "NULL path");
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(GB_ERR_ARG, std::string("cannot read ") + path);
    char line[512];
    int n = 0;
    std::map<std::string, Tile> add;
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        const char *colon = std::strchr(line, ':');
        if (!colon) continue;
        std::string key(line, size_t(colon - line));
        while (!key.empty() && key.back() == ' ') key.pop_back();
        Tile t;
        if (std::sscanf(colon + 1, "%d %d %d", &t.grid, &t.waves, &t.interleave) != 3 || t.grid < 1 ||
            (t.waves != gbd::kWaves && t.waves != 2 * gbd::kWaves)) {
            std::fclose(f);
            return fail(GB_ERR_ARG, "malformed tuning-cache line: " + std::string(line));
        }
        add[key] = t;
        ++n;
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_tile_mu);
    for (const auto &kv : add) g_tiles[kv.first] = kv.second;
    if (entries) *entries = n;
    return GB_OK;
}

void gb_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tiles.clear();
}

gb_status gb_batch_class_info(const gb_batch *b, int i, int64_t *info) {
    if (!b || !info) return fail(GB_ERR_ARG, "NULL argument");
    if (i < 0 || i >= int(b->classes.size())) return fail(GB_ERR_ARG, "class index out of range");
    const gb_batch::Class &c = b->classes[size_t(i)];
    info[0] = c.dim;
    info[1] = c.N;
    info[2] = c.prec;
    info[3] = c.nreq;
    info[4] = c.total;
    info[5] = c.grid;
    info[6] = c.solo ? 1 : 0;
    return GB_OK;
}

}  // extern "C"
