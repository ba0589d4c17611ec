// Host-side setup of the reference simplex element, mesh connectivity and
// SARK-4 coefficients.  Plain C++17, FP64, run once per mesh / time step size.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gbh {

// Row-major dense matrix.
struct Mat {
    int rows = 0, cols = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int r, int c) : rows(r), cols(c), a(size_t(r) * c, 0.0) {}
    double &operator()(int i, int j) { return a[size_t(i) * cols + j]; }
    double operator()(int i, int j) const { return a[size_t(i) * cols + j]; }
};

Mat matmul(const Mat &A, const Mat &B);
Mat transpose(const Mat &A);
Mat inverse(const Mat &A);  // partial-pivot LU; throws on singular

// Gauss-Jacobi rule (n points) for weight (1-x)^alpha (1+x)^beta, by the
// Golub-Welsch eigenvalue method on the Jacobi matrix.
void gauss_jacobi(int n, double alpha, double beta, std::vector<double> &x, std::vector<double> &w);

// Reference element of order N in dim dimensions (Section 3 of the paper).
struct RefElement {
    int dim = 2, N = 1, Np = 0, Nfaces = 0, Nfp = 0, Nc = 0, cub_degree = 0;
    std::vector<double> r;             // [Np][dim] Warp & Blend nodes
    Mat V;                             // orthonormal-basis Vandermonde [Np][Np]
    Mat D[3];                          // differentiation matrices [Np][Np]
    Mat M;                             // mass matrix
    std::vector<int> fmask;            // [Nfaces][Nfp]
    Mat LIFT;                          // [Np][Nfaces*Nfp], faces of measure 2
    Mat Icub;                          // [Nc][Np]
    Mat Pcub;                          // [Np][Nc]
    std::vector<double> cub_w;         // [Nc]
    std::vector<double> cub_r;         // [Nc][dim]
    Mat bary;                          // [Np][dim+1] P1 interpolation table
};

// Throws std::runtime_error for unsupported (dim, N).
RefElement build_ref_element(int dim, int N, int cub_degree);

// Element connectivity and trace map.
struct Connectivity {
    // vmapP[(e*Nfaces + f)*Nfp + i]: flat node index e'*Np + j' of the
    // exterior trace, or -1 (wall) / -2 (far field) for boundary faces.
    std::vector<int32_t> vmapP;
    std::vector<int32_t> etoe;         // [K][Nfaces], self for boundary
};

Connectivity build_connectivity(const RefElement &ref, int64_t nv, const double *vx, int64_t K,
                                const int32_t *etov, const double *period, const int8_t *face_tag,
                                std::string &err);

// Face-node index (f*Nfp + i) held by kernel face slot m.  The stage kernel
// gives slot 4 s + q to the lanes of quarter q of an element at step s.  On
// tetrahedra (four faces) slot m holds face m % 4, node m / 4, so each lane
// quarter keeps one face for all its steps; on triangles slots follow the
// face-node order.  Slots at or past Nfaces*Nfp are padding and map to
// themselves.
inline int slot_face_node(const RefElement &ref, int m) {
    const int nft = ref.Nfaces * ref.Nfp;
    if (m >= nft || ref.Nfaces != 4) return m;
    return (m % 4) * ref.Nfp + m / 4;
}

// Trace map in the device's blocked layout [ceil(K/16)][slots][16] (slots =
// Nfaces*Nfp rounded up to 4): the exterior node of the face node in kernel
// slot m (slot_face_node) of element e, or -1 (wall), -2 (far field), -3
// (padding of the last group or slot).
std::vector<int32_t> blocked_trace_map(const RefElement &ref, int64_t K, const Connectivity &conn);

// Consistency of the device tables of a mesh, checked on the host: every
// trace-map entry is a boundary code or a node of another element's face,
// the map is an involution on matched faces, the face-slot order is a
// permutation of the face nodes, the blocked copy equals the flat one in that
// order with padding where no element or slot exists, and every element's
// vertex ids are in range.  Returns an empty string or the first violation.
std::string check_mesh_tables(const RefElement &ref, int64_t nv, int64_t K, const int32_t *etov,
                              const Connectivity &conn, const std::vector<int32_t> &blocked);

// One member of a batched launch class, as the request table describes it:
// its element and vertex counts and the sizes in bytes of the device buffers
// its table entry points to.
struct BatchMemberLayout {
    int64_t K = 0, nv = 0;
    size_t etov_bytes = 0, vstage_bytes = 0, wstage_bytes = 0, vmap_bytes = 0, state_bytes = 0;
};

// Checks of a batched launch class before its table is uploaded: every
// buffer covers what the kernel addresses for that member (elements padded to
// whole groups of 16), the group offsets start at 0 and grow by each member's
// group count, the total stays below 2^31 groups, the member count within
// max_members, and the dynamic LDS the launch asks for within lds_limit.
std::string check_batch_class(int dim, int Np, int NF, int NFT, size_t elem_bytes,
                              const std::vector<BatchMemberLayout> &members, const std::vector<int32_t> &group_begin,
                              int64_t total_groups, int max_members, size_t lds_bytes, size_t lds_limit);

// SARK-4 coefficients for one field class with gamma = -dt * rate.
struct SarkCoef {
    double E[5];      // exp(c_i gamma) multiplying q_n: stages 0..3, final
    double a10, a20, a21, a30, a31, a32;
    double b[4];
};
SarkCoef sark_coefficients(double gamma);

}  // namespace gbh
