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

// SARK-4 coefficients for one field class with gamma = -dt * rate.
struct SarkCoef {
    double E[5];      // exp(c_i gamma) multiplying q_n: stages 0..3, final
    double a10, a20, a21, a30, a31, a32;
    double b[4];
};
SarkCoef sark_coefficients(double gamma);

}  // namespace gbh
