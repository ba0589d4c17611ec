// Host setup: reference element (Section 3 of the paper: nodal basis on
// Warp & Blend nodes, differentiation / lift / projection operators, cubature
// for the relaxation term), mesh connectivity with periodic matching, and the
// SARK-4 coefficients (Section 4) through the phi-functions of exponential
// integrators.
//
// Basis: the orthonormal collapsed-coordinate (Koornwinder-Dubiner) simplex
// polynomials, so the Vandermonde matrices stay well conditioned; mass matrix
// (V V^T)^-1; face mass matrices from the face Vandermonde matrices; Gauss
// rules by the Golub-Welsch method.
#include "host_ref.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>
#include <unordered_map>

namespace gbh {

// ---------------------------------------------------------------- linear algebra

Mat matmul(const Mat &A, const Mat &B) {
    if (A.cols != B.rows) throw std::runtime_error("matmul: shape");
    Mat C(A.rows, B.cols);
    for (int i = 0; i < A.rows; ++i)
        for (int k = 0; k < A.cols; ++k) {
            const double a = A(i, k);
            if (a == 0.0) continue;
            for (int j = 0; j < B.cols; ++j) C(i, j) += a * B(k, j);
        }
    return C;
}

Mat transpose(const Mat &A) {
    Mat T(A.cols, A.rows);
    for (int i = 0; i < A.rows; ++i)
        for (int j = 0; j < A.cols; ++j) T(j, i) = A(i, j);
    return T;
}

Mat inverse(const Mat &Ain) {
    const int n = Ain.rows;
    if (n != Ain.cols) throw std::runtime_error("inverse: not square");
    Mat A = Ain, X(n, n);
    for (int i = 0; i < n; ++i) X(i, i) = 1.0;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A(i, k)) > std::fabs(A(p, k))) p = i;
        if (A(p, k) == 0.0) throw std::runtime_error("inverse: singular");
        if (p != k)
            for (int j = 0; j < n; ++j) {
                std::swap(A(k, j), A(p, j));
                std::swap(X(k, j), X(p, j));
            }
        const double inv = 1.0 / A(k, k);
        for (int j = 0; j < n; ++j) {
            A(k, j) *= inv;
            X(k, j) *= inv;
        }
        for (int i = 0; i < n; ++i) {
            if (i == k) continue;
            const double f = A(i, k);
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A(i, j) -= f * A(k, j);
                X(i, j) -= f * X(k, j);
            }
        }
    }
    return X;
}

// Cyclic Jacobi eigenvalue iteration for a small symmetric matrix.
static void sym_eig(Mat A, std::vector<double> &ev, Mat &Q) {
    const int n = A.rows;
    Q = Mat(n, n);
    for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
        if (off < 1e-34) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (std::fabs(A(p, q)) < 1e-300) continue;
                const double theta = (A(q, q) - A(p, p)) / (2.0 * A(p, q));
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q(k, p), qkq = Q(k, q);
                    Q(k, p) = c * qkp - s * qkq;
                    Q(k, q) = s * qkp + c * qkq;
                }
            }
    }
    ev.resize(n);
    for (int i = 0; i < n; ++i) ev[i] = A(i, i);
}

// ---------------------------------------------------------------- Jacobi polynomials

// Orthonormal Jacobi polynomial P_n^{(alpha,beta)} at x (unit norm with the
// weight (1-x)^alpha (1+x)^beta on [-1,1]), by the three-term recurrence.
static double jacobi_p(double x, double alpha, double beta, int n) {
    const double ab = alpha + beta;
    const double g0 = std::pow(2.0, ab + 1.0) / (ab + 1.0) * std::tgamma(alpha + 1.0) *
                      std::tgamma(beta + 1.0) / std::tgamma(ab + 1.0);
    double p0 = 1.0 / std::sqrt(g0);
    if (n == 0) return p0;
    const double g1 = (alpha + 1.0) * (beta + 1.0) / (ab + 3.0) * g0;
    double p1 = ((ab + 2.0) * x / 2.0 + (alpha - beta) / 2.0) / std::sqrt(g1);
    if (n == 1) return p1;
    double aold = 2.0 / (2.0 + ab) * std::sqrt((alpha + 1.0) * (beta + 1.0) / (ab + 3.0));
    for (int i = 1; i < n; ++i) {
        const double h1 = 2.0 * i + ab;
        const double anew = 2.0 / (h1 + 2.0) *
                            std::sqrt((i + 1.0) * (i + 1.0 + ab) * (i + 1.0 + alpha) * (i + 1.0 + beta) /
                                      (h1 + 1.0) / (h1 + 3.0));
        const double bnew = -(alpha * alpha - beta * beta) / h1 / (h1 + 2.0);
        const double p2 = (-aold * p0 + (x - bnew) * p1) / anew;
        p0 = p1;
        p1 = p2;
        aold = anew;
    }
    return p1;
}

static double grad_jacobi_p(double x, double alpha, double beta, int n) {
    if (n == 0) return 0.0;
    return std::sqrt(n * (n + alpha + beta + 1.0)) * jacobi_p(x, alpha + 1.0, beta + 1.0, n - 1);
}

void gauss_jacobi(int n, double alpha, double beta, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double ab = alpha + beta;
    const double mu0 = std::pow(2.0, ab + 1.0) / (ab + 1.0) * std::tgamma(alpha + 1.0) *
                       std::tgamma(beta + 1.0) / std::tgamma(ab + 1.0);
    if (n == 1) {
        x[0] = -(alpha - beta) / (ab + 2.0);
        w[0] = mu0;
        return;
    }
    Mat J(n, n);
    for (int i = 0; i < n; ++i) {
        const double h1 = 2.0 * i + ab;
        J(i, i) = (ab < 1e-14 && i == 0) ? 0.0 : -(alpha * alpha - beta * beta) / (h1 + 2.0) / h1;
        if (i + 1 < n) {
            const double k = i + 1.0;
            const double b = 2.0 / (h1 + 2.0) *
                             std::sqrt(k * (k + ab) * (k + alpha) * (k + beta) / (h1 + 1.0) / (h1 + 3.0));
            J(i, i + 1) = J(i + 1, i) = b;
        }
    }
    std::vector<double> ev;
    Mat Q;
    sym_eig(J, ev, Q);
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return ev[a] < ev[b]; });
    for (int i = 0; i < n; ++i) {
        x[i] = ev[idx[i]];
        w[i] = Q(0, idx[i]) * Q(0, idx[i]) * mu0;
    }
}

static std::vector<double> gauss_lobatto(int N) {
    std::vector<double> r(N + 1);
    r[0] = -1.0;
    r[N] = 1.0;
    if (N >= 2) {
        std::vector<double> x, w;
        gauss_jacobi(N - 1, 1.0, 1.0, x, w);
        for (int i = 0; i < N - 1; ++i) r[i + 1] = x[i];
    }
    return r;
}

// ---------------------------------------------------------------- Warp & Blend nodes

// warp(r)/(1-r^2) with warp the interpolant, on equispaced nodes, of the
// displacement from equispaced to Gauss-Lobatto nodes (Warburton 2006).  The
// interpolant is formed through the Legendre Vandermonde matrix.
static std::vector<double> warp_factor(int N, const std::vector<double> &rout) {
    const std::vector<double> lgl = gauss_lobatto(N);
    std::vector<double> req(N + 1);
    for (int i = 0; i <= N; ++i) req[i] = -1.0 + 2.0 * i / N;
    Mat Veq(N + 1, N + 1);
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) Veq(i, j) = jacobi_p(req[i], 0, 0, j);
    // coefficients c of the interpolant: Veq c = lgl - req
    const Mat Vi = inverse(Veq);
    std::vector<double> coef(N + 1, 0.0);
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) coef[j] += Vi(j, i) * (lgl[i] - req[i]);
    std::vector<double> out(rout.size());
    for (size_t p = 0; p < rout.size(); ++p) {
        double wv = 0.0;
        for (int j = 0; j <= N; ++j) wv += coef[j] * jacobi_p(rout[p], 0, 0, j);
        const double r = rout[p];
        out[p] = (std::fabs(r) < 1.0 - 1e-10) ? wv / (1.0 - r * r) : 0.0;
    }
    return out;
}

// Displacement in the equilateral triangle with barycentric (L1, L2, L3).
static void equilateral_shift(int N, double alpha, const std::vector<double> &L1, const std::vector<double> &L2,
                              const std::vector<double> &L3, std::vector<double> &dx, std::vector<double> &dy) {
    const size_t n = L1.size();
    std::vector<double> a(n), b(n), c(n);
    for (size_t i = 0; i < n; ++i) {
        a[i] = L3[i] - L2[i];
        b[i] = L1[i] - L3[i];
        c[i] = L2[i] - L1[i];
    }
    const auto w1 = warp_factor(N, a), w2 = warp_factor(N, b), w3 = warp_factor(N, c);
    dx.assign(n, 0.0);
    dy.assign(n, 0.0);
    const double c2 = std::cos(2 * M_PI / 3), s2 = std::sin(2 * M_PI / 3);
    const double c4 = std::cos(4 * M_PI / 3), s4 = std::sin(4 * M_PI / 3);
    for (size_t i = 0; i < n; ++i) {
        const double W1 = 4 * L2[i] * L3[i] * w1[i] * (1 + (alpha * L1[i]) * (alpha * L1[i]));
        const double W2 = 4 * L1[i] * L3[i] * w2[i] * (1 + (alpha * L2[i]) * (alpha * L2[i]));
        const double W3 = 4 * L1[i] * L2[i] * w3[i] * (1 + (alpha * L3[i]) * (alpha * L3[i]));
        dx[i] = W1 + c2 * W2 + c4 * W3;
        dy[i] = s2 * W2 + s4 * W3;
    }
}

static const double kAlphaTri[15] = {0.0000, 0.0000, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
                                     1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258};
static const double kAlphaTet[15] = {0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577,
                                     1.1603, 1.10153, 0.6080, 0.4523, 0.8856, 0.8717, 0.9655};

static std::vector<double> nodes_tri(int N) {
    const double alpha = N <= 15 ? kAlphaTri[N - 1] : 5.0 / 3.0;
    std::vector<double> L1, L2, L3;
    for (int n = 0; n <= N; ++n)
        for (int m = 0; m <= N - n; ++m) {
            L1.push_back(double(n) / N);
            L3.push_back(double(m) / N);
            L2.push_back(1.0 - L1.back() - L3.back());
        }
    std::vector<double> dx, dy;
    equilateral_shift(N, alpha, L1, L2, L3, dx, dy);
    const size_t Np = L1.size();
    std::vector<double> rs(2 * Np);
    const double s3 = std::sqrt(3.0);
    for (size_t i = 0; i < Np; ++i) {
        const double x = -L2[i] + L3[i] + dx[i];
        const double y = (-L2[i] - L3[i] + 2 * L1[i]) / s3 + dy[i];
        const double B1 = (s3 * y + 1.0) / 3.0;
        const double B2 = (-3.0 * x - s3 * y + 2.0) / 6.0;
        const double B3 = (3.0 * x - s3 * y + 2.0) / 6.0;
        rs[2 * i] = -B2 + B3 - B1;
        rs[2 * i + 1] = -B2 - B3 + B1;
    }
    return rs;
}

static std::vector<double> nodes_tet(int N) {
    const double alpha = N <= 15 ? kAlphaTet[N - 1] : 1.0;
    const double tol = 1e-10;
    std::vector<double> L1, L2, L3, L4;
    for (int n = 0; n <= N; ++n)
        for (int m = 0; m <= N - n; ++m)
            for (int q = 0; q <= N - n - m; ++q) {
                const double r = -1.0 + 2.0 * q / N, s = -1.0 + 2.0 * m / N, t = -1.0 + 2.0 * n / N;
                L1.push_back((1 + t) / 2);
                L2.push_back((1 + s) / 2);
                L3.push_back(-(1 + r + s + t) / 2);
                L4.push_back((1 + r) / 2);
            }
    const size_t Np = L1.size();
    const double v1[3] = {-1.0, -1 / std::sqrt(3.0), -1 / std::sqrt(6.0)};
    const double v2[3] = {1.0, -1 / std::sqrt(3.0), -1 / std::sqrt(6.0)};
    const double v3[3] = {0.0, 2 / std::sqrt(3.0), -1 / std::sqrt(6.0)};
    const double v4[3] = {0.0, 0.0, 3 / std::sqrt(6.0)};
    double t1[4][3], t2[4][3];
    for (int d = 0; d < 3; ++d) {
        t1[0][d] = v2[d] - v1[d];
        t1[1][d] = v2[d] - v1[d];
        t1[2][d] = v3[d] - v2[d];
        t1[3][d] = v3[d] - v1[d];
        t2[0][d] = v3[d] - 0.5 * (v1[d] + v2[d]);
        t2[1][d] = v4[d] - 0.5 * (v1[d] + v2[d]);
        t2[2][d] = v4[d] - 0.5 * (v2[d] + v3[d]);
        t2[3][d] = v4[d] - 0.5 * (v1[d] + v3[d]);
    }
    for (int f = 0; f < 4; ++f) {
        double n1 = 0, n2 = 0;
        for (int d = 0; d < 3; ++d) {
            n1 += t1[f][d] * t1[f][d];
            n2 += t2[f][d] * t2[f][d];
        }
        for (int d = 0; d < 3; ++d) {
            t1[f][d] /= std::sqrt(n1);
            t2[f][d] /= std::sqrt(n2);
        }
    }
    std::vector<double> X(3 * Np), shift(3 * Np, 0.0);
    for (size_t i = 0; i < Np; ++i)
        for (int d = 0; d < 3; ++d) X[3 * i + d] = L3[i] * v1[d] + L4[i] * v2[d] + L2[i] * v3[d] + L1[i] * v4[d];
    for (int f = 0; f < 4; ++f) {
        const std::vector<double> *La, *Lb, *Lc, *Ld;
        if (f == 0) { La = &L1; Lb = &L2; Lc = &L3; Ld = &L4; }
        else if (f == 1) { La = &L2; Lb = &L1; Lc = &L3; Ld = &L4; }
        else if (f == 2) { La = &L3; Lb = &L1; Lc = &L4; Ld = &L2; }
        else { La = &L4; Lb = &L1; Lc = &L3; Ld = &L2; }
        std::vector<double> w1, w2;
        equilateral_shift(N, alpha, *Lb, *Lc, *Ld, w1, w2);
        for (size_t i = 0; i < Np; ++i) {
            const double la = (*La)[i], lb = (*Lb)[i], lc = (*Lc)[i], ld = (*Ld)[i];
            double blend = lb * lc * ld;
            const double denom = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la);
            if (denom > tol) blend = (1 + (alpha * la) * (alpha * la)) * blend / denom;
            for (int d = 0; d < 3; ++d) shift[3 * i + d] += blend * w1[i] * t1[f][d] + blend * w2[i] * t2[f][d];
            const int npos = (lb > tol) + (lc > tol) + (ld > tol);
            if (la < tol && npos < 3)
                for (int d = 0; d < 3; ++d) shift[3 * i + d] = w1[i] * t1[f][d] + w2[i] * t2[f][d];
        }
    }
    // equilateral -> reference right tetrahedron
    Mat A(3, 3);
    for (int d = 0; d < 3; ++d) {
        A(d, 0) = 0.5 * (v2[d] - v1[d]);
        A(d, 1) = 0.5 * (v3[d] - v1[d]);
        A(d, 2) = 0.5 * (v4[d] - v1[d]);
    }
    const Mat Ai = inverse(A);
    std::vector<double> rst(3 * Np);
    for (size_t i = 0; i < Np; ++i) {
        double rhs[3];
        for (int d = 0; d < 3; ++d) rhs[d] = X[3 * i + d] + shift[3 * i + d] - 0.5 * (v2[d] + v3[d] + v4[d] - v1[d]);
        for (int a = 0; a < 3; ++a) rst[3 * i + a] = Ai(a, 0) * rhs[0] + Ai(a, 1) * rhs[1] + Ai(a, 2) * rhs[2];
    }
    return rst;
}

// ---------------------------------------------------------------- orthonormal simplex basis

// Value and reference gradient of basis function (i, j) on the triangle.
static void simplex2d(double r, double s, int i, int j, double &v, double &dr, double &ds) {
    const double a = (s != 1.0) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
    const double b = s;
    const double fa = jacobi_p(a, 0, 0, i), dfa = grad_jacobi_p(a, 0, 0, i);
    const double gb = jacobi_p(b, 2 * i + 1, 0, j), dgb = grad_jacobi_p(b, 2 * i + 1, 0, j);
    v = std::sqrt(2.0) * fa * gb * std::pow(1.0 - b, i);
    double ddr = dfa * gb;
    if (i > 0) ddr *= std::pow(0.5 * (1 - b), i - 1);
    double dds = dfa * (gb * (0.5 * (1 + a)));
    if (i > 0) dds *= std::pow(0.5 * (1 - b), i - 1);
    double tmp = dgb * std::pow(0.5 * (1 - b), i);
    if (i > 0) tmp -= 0.5 * i * gb * std::pow(0.5 * (1 - b), i - 1);
    dds += fa * tmp;
    const double nrm = std::pow(2.0, i + 0.5);
    dr = ddr * nrm;
    ds = dds * nrm;
}

// Value and reference gradient of basis function (i, j, k) on the tetrahedron.
static void simplex3d(double r, double s, double t, int i, int j, int k, double &v, double &dr, double &ds,
                      double &dt) {
    const double a = (s + t != 0.0) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
    const double b = (t != 1.0) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
    const double c = t;
    const double fa = jacobi_p(a, 0, 0, i), dfa = grad_jacobi_p(a, 0, 0, i);
    const double gb = jacobi_p(b, 2 * i + 1, 0, j), dgb = grad_jacobi_p(b, 2 * i + 1, 0, j);
    const double hc = jacobi_p(c, 2 * (i + j) + 2, 0, k), dhc = grad_jacobi_p(c, 2 * (i + j) + 2, 0, k);
    v = 2.0 * std::sqrt(2.0) * fa * gb * std::pow(1.0 - b, i) * hc * std::pow(1.0 - c, i + j);
    double vr = dfa * (gb * hc);
    if (i > 0) vr *= std::pow(0.5 * (1 - b), i - 1);
    if (i + j > 0) vr *= std::pow(0.5 * (1 - c), i + j - 1);
    double vs = 0.5 * (1 + a) * vr;
    double tmp = dgb * std::pow(0.5 * (1 - b), i);
    if (i > 0) tmp += (-0.5 * i) * (gb * std::pow(0.5 * (1 - b), i - 1));
    if (i + j > 0) tmp *= std::pow(0.5 * (1 - c), i + j - 1);
    tmp = fa * (tmp * hc);
    vs += tmp;
    double vt = 0.5 * (1 + a) * vr + 0.5 * (1 + b) * tmp;
    tmp = dhc * std::pow(0.5 * (1 - c), i + j);
    if (i + j > 0) tmp -= 0.5 * (i + j) * (hc * std::pow(0.5 * (1 - c), i + j - 1));
    tmp = fa * (gb * tmp);
    tmp *= std::pow(0.5 * (1 - b), i);
    vt += tmp;
    const double nrm = std::pow(2.0, 2 * i + j + 1.5);
    dr = vr * nrm;
    ds = vs * nrm;
    dt = vt * nrm;
}

// Vandermonde matrix (and gradients) of the dim-D basis at points pts [n][dim].
static void vandermonde(int dim, int N, const std::vector<double> &pts, Mat &V, Mat *G) {
    const int n = int(pts.size()) / dim;
    std::vector<std::array<int, 3>> ex;
    if (dim == 2) {
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N - i; ++j) ex.push_back({i, j, 0});
    } else {
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N - i; ++j)
                for (int k = 0; k <= N - i - j; ++k) ex.push_back({i, j, k});
    }
    const int Np = int(ex.size());
    V = Mat(n, Np);
    if (G)
        for (int d = 0; d < dim; ++d) G[d] = Mat(n, Np);
    for (int p = 0; p < n; ++p)
        for (int m = 0; m < Np; ++m) {
            double v, gr, gs, gt = 0.0;
            if (dim == 2)
                simplex2d(pts[2 * p], pts[2 * p + 1], ex[m][0], ex[m][1], v, gr, gs);
            else
                simplex3d(pts[3 * p], pts[3 * p + 1], pts[3 * p + 2], ex[m][0], ex[m][1], ex[m][2], v, gr, gs, gt);
            V(p, m) = v;
            if (G) {
                G[0](p, m) = gr;
                G[1](p, m) = gs;
                if (dim == 3) G[2](p, m) = gt;
            }
        }
}

static void cubature_rule(int dim, int degree, std::vector<double> &pts, std::vector<double> &w) {
    const int n = (degree + 2) / 2;
    std::vector<double> a, wa, b, wb, c, wc;
    gauss_jacobi(n, 0, 0, a, wa);
    gauss_jacobi(n, 1, 0, b, wb);
    pts.clear();
    w.clear();
    if (dim == 2) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                pts.push_back((1 + a[i]) * (1 - b[j]) / 2 - 1);
                pts.push_back(b[j]);
                w.push_back(wa[i] * wb[j] / 2);
            }
        return;
    }
    gauss_jacobi(n, 2, 0, c, wc);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                pts.push_back((1 + a[i]) * (1 - b[j]) * (1 - c[k]) / 4 - 1);
                pts.push_back((1 + b[j]) * (1 - c[k]) / 2 - 1);
                pts.push_back(c[k]);
                w.push_back(wa[i] * wb[j] * wc[k] / 8);
            }
}

RefElement build_ref_element(int dim, int N, int cub_degree) {
    if (!((dim == 2 && N >= 1 && N <= 8) || (dim == 3 && N >= 1 && N <= 5)))
        throw std::runtime_error("unsupported (dim, N)");
    RefElement R;
    R.dim = dim;
    R.N = N;
    R.Np = dim == 2 ? (N + 1) * (N + 2) / 2 : (N + 1) * (N + 2) * (N + 3) / 6;
    R.Nfaces = dim + 1;
    R.Nfp = dim == 2 ? N + 1 : (N + 1) * (N + 2) / 2;
    R.r = dim == 2 ? nodes_tri(N) : nodes_tet(N);
    const int Np = R.Np;
    Mat G[3];
    vandermonde(dim, N, R.r, R.V, G);
    const Mat Vi = inverse(R.V);
    for (int d = 0; d < dim; ++d) R.D[d] = matmul(G[d], Vi);
    R.M = inverse(matmul(R.V, transpose(R.V)));
    // barycentric table and face masks
    R.bary = Mat(Np, dim + 1);
    for (int i = 0; i < Np; ++i) {
        const double *x = &R.r[dim * i];
        if (dim == 2) {
            R.bary(i, 0) = -(x[0] + x[1]) / 2;
            R.bary(i, 1) = (1 + x[0]) / 2;
            R.bary(i, 2) = (1 + x[1]) / 2;
        } else {
            R.bary(i, 0) = -(1 + x[0] + x[1] + x[2]) / 2;
            R.bary(i, 1) = (1 + x[0]) / 2;
            R.bary(i, 2) = (1 + x[1]) / 2;
            R.bary(i, 3) = (1 + x[2]) / 2;
        }
    }
    // face f is opposite to vertex: triangle faces (0,1),(1,2),(2,0) are
    // opposite vertices 2,0,1; tetrahedron faces (0,1,2),(0,1,3),(1,2,3),(0,2,3)
    // are opposite vertices 3,2,0,1
    const int opp2[3] = {2, 0, 1}, opp3[4] = {3, 2, 0, 1};
    for (int f = 0; f < R.Nfaces; ++f) {
        const int ov = dim == 2 ? opp2[f] : opp3[f];
        int cnt = 0;
        for (int i = 0; i < Np; ++i)
            if (std::fabs(R.bary(i, ov)) < 1e-10) {
                R.fmask.push_back(i);
                ++cnt;
            }
        if (cnt != R.Nfp) throw std::runtime_error("face mask size");
    }
    // face mass matrices from the face Vandermonde matrices (measure 2)
    Mat E(Np, R.Nfaces * R.Nfp);
    for (int f = 0; f < R.Nfaces; ++f) {
        std::vector<double> fp;
        for (int m = 0; m < R.Nfp; ++m) {
            const double *x = &R.r[dim * R.fmask[f * R.Nfp + m]];
            if (dim == 2) {
                fp.push_back(f == 2 ? x[1] : x[0]);
            } else {
                if (f == 0) { fp.push_back(x[0]); fp.push_back(x[1]); }
                else if (f == 1) { fp.push_back(x[0]); fp.push_back(x[2]); }
                else { fp.push_back(x[1]); fp.push_back(x[2]); }
            }
        }
        Mat Vf;
        if (dim == 2) {
            Vf = Mat(R.Nfp, R.Nfp);
            for (int m = 0; m < R.Nfp; ++m)
                for (int k = 0; k <= N; ++k) Vf(m, k) = jacobi_p(fp[m], 0, 0, k);
        } else {
            vandermonde(2, N, fp, Vf, nullptr);
        }
        const Mat Mf = inverse(matmul(Vf, transpose(Vf)));
        for (int m = 0; m < R.Nfp; ++m)
            for (int l = 0; l < R.Nfp; ++l) E(R.fmask[f * R.Nfp + m], f * R.Nfp + l) = Mf(m, l);
    }
    R.LIFT = matmul(R.V, matmul(transpose(R.V), E));
    // cubature
    R.cub_degree = cub_degree > 0 ? cub_degree : 3 * N;
    if (R.cub_degree < 2 * N) throw std::runtime_error("cubature degree below 2N");
    cubature_rule(dim, R.cub_degree, R.cub_r, R.cub_w);
    R.Nc = int(R.cub_w.size());
    Mat Vc;
    vandermonde(dim, N, R.cub_r, Vc, nullptr);
    R.Icub = matmul(Vc, Vi);
    Mat IW = transpose(R.Icub);
    for (int i = 0; i < Np; ++i)
        for (int k = 0; k < R.Nc; ++k) IW(i, k) *= R.cub_w[k];
    R.Pcub = matmul(matmul(R.V, transpose(R.V)), IW);
    return R;
}

// ---------------------------------------------------------------- connectivity

namespace {
struct FaceKey {
    std::array<int64_t, 12> k{};
    bool operator==(const FaceKey &o) const { return k == o.k; }
};
struct FaceKeyHash {
    size_t operator()(const FaceKey &f) const {
        uint64_t h = 1469598103934665603ull;
        for (int64_t v : f.k) {
            h ^= uint64_t(v);
            h *= 1099511628211ull;
        }
        return size_t(h);
    }
};
}  // namespace

Connectivity build_connectivity(const RefElement &R, int64_t nv, const double *vx, int64_t K, const int32_t *etov,
                                const double *period, const int8_t *face_tag, std::string &err) {
    const int dim = R.dim, nvert = dim + 1, Nf = R.Nfaces, Nfp = R.Nfp, Np = R.Np;
    Connectivity C;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, P[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        lo[d] = 1e300;
        hi[d] = -1e300;
        P[d] = period ? period[d] : 0.0;
    }
    for (int64_t v = 0; v < nv; ++v)
        for (int d = 0; d < dim; ++d) {
            lo[d] = std::min(lo[d], vx[v * dim + d]);
            hi[d] = std::max(hi[d], vx[v * dim + d]);
        }
    double scale = 1.0;
    for (int d = 0; d < dim; ++d) scale = std::max(scale, hi[d] - lo[d]);
    auto wrap = [&](double x, int d) {
        if (P[d] <= 0) return x;
        double y = std::fmod(x - lo[d], P[d]);
        if (y < 0) y += P[d];
        if (std::fabs(y - P[d]) < 1e-9 * P[d]) y = 0.0;
        return y + lo[d];
    };
    auto quant = [&](double x) { return int64_t(std::llround(x / scale * 1e8)); };
    const int fv2[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    const int fv3[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
    std::unordered_map<FaceKey, int64_t, FaceKeyHash> open;
    open.reserve(size_t(K) * Nf);
    C.etoe.assign(size_t(K) * Nf, -1);
    std::vector<int32_t> etof(size_t(K) * Nf, -1);
    for (int64_t e = 0; e < K; ++e) {
        for (int f = 0; f < Nf; ++f) {
            const int nfv = dim;
            FaceKey key;
            double cen[3] = {0, 0, 0};
            std::array<std::array<int64_t, 3>, 3> pts{};
            for (int a = 0; a < nfv; ++a) {
                const int lv = dim == 2 ? fv2[f][a] : fv3[f][a];
                const int32_t gv = etov[e * nvert + lv];
                if (gv < 0 || gv >= nv) {
                    err = "etov index out of range";
                    return C;
                }
                for (int d = 0; d < dim; ++d) {
                    cen[d] += vx[int64_t(gv) * dim + d] / nfv;
                    pts[a][d] = quant(wrap(vx[int64_t(gv) * dim + d], d));
                }
            }
            std::sort(pts.begin(), pts.begin() + nfv);
            for (int d = 0; d < dim; ++d) key.k[d] = quant(wrap(cen[d], d));
            for (int a = 0; a < nfv; ++a)
                for (int d = 0; d < 3; ++d) key.k[3 + 3 * a + d] = pts[a][d];
            auto it = open.find(key);
            if (it != open.end()) {
                const int64_t other = it->second;
                const int64_t e2 = other / Nf;
                const int f2 = int(other % Nf);
                C.etoe[e * Nf + f] = int32_t(e2);
                etof[e * Nf + f] = f2;
                C.etoe[e2 * Nf + f2] = int32_t(e);
                etof[e2 * Nf + f2] = f;
                open.erase(it);
            } else {
                open.emplace(key, e * Nf + f);
            }
        }
    }
    // node coordinates of face nodes on the initial mesh
    auto node_x = [&](int64_t e, int i, double *x) {
        for (int d = 0; d < dim; ++d) {
            x[d] = 0.0;
            for (int v = 0; v < nvert; ++v) x[d] += R.bary(i, v) * vx[int64_t(etov[e * nvert + v]) * dim + d];
        }
    };
    C.vmapP.assign(size_t(K) * Nf * Nfp, 0);
    std::vector<double> xnb(size_t(Nfp) * 3);
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < Nf; ++f) {
            const int64_t e2 = C.etoe[e * Nf + f];
            int32_t *out = &C.vmapP[(e * Nf + f) * Nfp];
            if (e2 < 0) {
                const int tag = face_tag ? face_tag[e * Nf + f] : 0;
                if (tag != 1 && tag != 2) {
                    err = "unmatched face without a wall / far-field tag";
                    return C;
                }
                C.etoe[e * Nf + f] = int32_t(e);
                for (int m = 0; m < Nfp; ++m) out[m] = tag == 1 ? -1 : -2;
                continue;
            }
            const int f2 = etof[e * Nf + f];
            // the neighbour face's node coordinates, once per face
            for (int l = 0; l < Nfp; ++l) node_x(e2, R.fmask[f2 * Nfp + l], &xnb[size_t(l) * 3]);
            for (int m = 0; m < Nfp; ++m) {
                double xa[3];
                node_x(e, R.fmask[f * Nfp + m], xa);
                double best = 1e300;
                int bj = -1;
                for (int l = 0; l < Nfp; ++l) {
                    const double *xb = &xnb[size_t(l) * 3];
                    double d2 = 0.0;
                    for (int d = 0; d < dim; ++d) {
                        double dd = xa[d] - xb[d];
                        if (P[d] > 0) dd -= P[d] * std::nearbyint(dd / P[d]);
                        d2 += dd * dd;
                    }
                    if (d2 < best) {
                        best = d2;
                        bj = l;
                    }
                }
                if (std::sqrt(best) > 1e-8 * scale) {
                    err = "face nodes do not match";
                    return C;
                }
                const int64_t flat = e2 * Np + R.fmask[f2 * Nfp + bj];
                if (flat > INT32_MAX) {
                    err = "mesh too large for 32-bit node indices";
                    return C;
                }
                out[m] = int32_t(flat);
            }
        }
    return C;
}

// ---------------------------------------------------------------- table checks

std::vector<int32_t> blocked_trace_map(const RefElement &ref, int64_t K, const Connectivity &conn) {
    const int NFT = ref.Nfaces * ref.Nfp;
    const int slots = (NFT + 3) / 4 * 4;
    const int64_t G = (K + 15) / 16;
    std::vector<int32_t> blk(size_t(G) * slots * 16, -3);
    for (int64_t e = 0; e < K; ++e)
        for (int m = 0; m < NFT; ++m)
            blk[((e >> 4) * slots + m) * 16 + (e & 15)] = conn.vmapP[e * NFT + slot_face_node(ref, m)];
    return blk;
}

std::string check_mesh_tables(const RefElement &ref, int64_t nv, int64_t K, const int32_t *etov,
                              const Connectivity &conn, const std::vector<int32_t> &blocked) {
    const int Np = ref.Np, Nf = ref.Nfaces, Nfp = ref.Nfp, NFT = Nf * Nfp, nvert = ref.dim + 1;
    const int slots = (NFT + 3) / 4 * 4;
    const int64_t G = (K + 15) / 16;
    if (int64_t(conn.vmapP.size()) != K * NFT) return "trace map has the wrong size";
    if (int64_t(blocked.size()) != G * slots * 16) return "blocked trace map has the wrong size";
    // the kernel's face-slot order visits every face node once
    std::vector<char> seen(size_t(NFT), 0);
    for (int m = 0; m < NFT; ++m) {
        const int fn = slot_face_node(ref, m);
        if (fn < 0 || fn >= NFT || seen[size_t(fn)]++) return "face-slot order is not a permutation of the face nodes";
    }
    for (int64_t e = 0; e < K; ++e)
        for (int v = 0; v < nvert; ++v) {
            const int32_t gv = etov[e * nvert + v];
            if (gv < 0 || gv >= nv) return "vertex id out of range at element " + std::to_string(e);
        }
    // node -> (face slot) of each element, for the involution check
    std::vector<int> slot_of_node(size_t(Nf) * Np, -1);
    for (int f = 0; f < Nf; ++f)
        for (int m = 0; m < Nfp; ++m) slot_of_node[size_t(f) * Np + ref.fmask[f * Nfp + m]] = f * Nfp + m;
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < Nf; ++f)
            for (int m = 0; m < Nfp; ++m) {
                const int32_t idx = conn.vmapP[(e * Nf + f) * Nfp + m];
                if (idx == -1 || idx == -2) continue;
                if (idx < 0 || int64_t(idx) >= K * Np)
                    return "trace-map entry out of range at element " + std::to_string(e);
                const int64_t e2 = idx / Np;
                const int j2 = int(idx - e2 * Np);
                // the partner's node lies on the face that points back at e
                int back = -1;
                for (int ff = 0; ff < Nf; ++ff)
                    if (conn.etoe[e2 * Nf + ff] == e && slot_of_node[size_t(ff) * Np + j2] >= 0) {
                        const int m2 = slot_of_node[size_t(ff) * Np + j2];
                        if (conn.vmapP[e2 * NFT + m2] == int32_t(e * Np + ref.fmask[f * Nfp + m])) back = m2;
                    }
                if (back < 0) return "trace map is not an involution at element " + std::to_string(e);
            }
    for (int64_t g = 0; g < G; ++g)
        for (int m = 0; m < slots; ++m)
            for (int l = 0; l < 16; ++l) {
                const int64_t e = g * 16 + l;
                const int32_t got = blocked[(g * slots + m) * 16 + l];
                const int32_t want = (e < K && m < NFT) ? conn.vmapP[e * NFT + slot_face_node(ref, m)] : -3;
                if (got != want) return "blocked trace map differs from the flat one at group " + std::to_string(g);
            }
    return std::string();
}

std::string check_batch_class(int dim, int Np, int NF, int NFT, size_t elem_bytes,
                              const std::vector<BatchMemberLayout> &members, const std::vector<int32_t> &group_begin,
                              int64_t total_groups, int max_members, size_t lds_bytes, size_t lds_limit) {
    if (members.empty()) return "empty class";
    if (int(members.size()) > max_members) return "more members than the request table holds";
    if (group_begin.size() != members.size()) return "group offsets and members differ in number";
    const int slots = (NFT + 3) / 4 * 4;
    int64_t g = 0;
    for (size_t i = 0; i < members.size(); ++i) {
        const BatchMemberLayout &b = members[i];
        const int64_t groups = (b.K + 15) / 16;
        if (b.K <= 0 || b.nv <= 0) return "member " + std::to_string(i) + " is empty";
        if (group_begin[i] != g) return "group offset of member " + std::to_string(i) + " is not the running sum";
        if (b.etov_bytes < size_t(b.K) * (dim + 1) * sizeof(int32_t)) return "vertex-id buffer too small";
        if (b.vstage_bytes < 5 * size_t(b.nv) * dim * sizeof(double)) return "stage-position buffer too small";
        if (b.wstage_bytes < 4 * size_t(b.nv) * dim * sizeof(double)) return "stage-velocity buffer too small";
        if (b.vmap_bytes < size_t(groups) * slots * 16 * sizeof(int32_t)) return "trace-map buffer too small";
        if (b.state_bytes < size_t(groups) * 16 * NF * Np * elem_bytes) return "state buffer too small";
        g += groups;
    }
    if (g != total_groups) return "total group count differs from the members' sum";
    if (total_groups >= (int64_t(1) << 31)) return "too many element groups in one class";
    if (lds_bytes > lds_limit) return "dynamic LDS of the launch exceeds the limit set for the kernel";
    return std::string();
}

// ---------------------------------------------------------------- SARK-4

// phi_k(z) = sum_m z^m / (m+k)!  (k = 1..3): power series for |z| < 1, the
// recurrence phi_{k+1} = (phi_k - 1/k!)/z otherwise.
static void phi123(double z, double &p1, double &p2, double &p3) {
    if (std::fabs(z) < 1.0) {
        p1 = p2 = p3 = 0.0;
        double term = 1.0;  // z^m
        double f1 = 1.0, f2 = 0.5, f3 = 1.0 / 6.0;  // 1/(m+k)!
        for (int m = 0; m < 40; ++m) {
            p1 += term * f1;
            p2 += term * f2;
            p3 += term * f3;
            term *= z;
            f1 /= (m + 2);
            f2 /= (m + 3);
            f3 /= (m + 4);
        }
        return;
    }
    p1 = std::expm1(z) / z;
    p2 = (p1 - 1.0) / z;
    p3 = (p2 - 0.5) / z;
}

SarkCoef sark_coefficients(double g) {
    SarkCoef c{};
    double h1, h2, h3, f1, f2, f3;
    phi123(0.5 * g, h1, h2, h3);
    phi123(g, f1, f2, f3);
    c.E[0] = 1.0;
    c.E[1] = c.E[2] = std::exp(0.5 * g);
    c.E[3] = c.E[4] = std::exp(g);
    c.a10 = 0.5 * h1;
    c.a20 = 0.5 * h1 - h2;
    c.a21 = h2;
    c.a30 = f1 - 2.0 * f2;
    c.a31 = 0.0;
    c.a32 = 2.0 * f2;
    c.b[0] = f1 - 3.0 * f2 + 4.0 * f3;
    c.b[1] = c.b[2] = 2.0 * f2 - 4.0 * f3;
    c.b[3] = 4.0 * f3 - f2;
    return c;
}

}  // namespace gbh
