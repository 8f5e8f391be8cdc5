// Host-side set-up of an instance: the ordinate set and the initial low-rank
// factors.  Runs once per dlr_create; nothing here is part of the time step.
#include "host_setup.h"

#include <cmath>
#include <stdexcept>

namespace dlr {

namespace {
constexpr double kPi = 3.14159265358979323846;
}

// n-point Gauss-Legendre nodes/weights on (-1, 1): Newton's method on P_n from
// the Chebyshev-like initial guess cos(pi (i + 3/4) / (n + 1/2)), with P_n and
// P_n' from the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // one more evaluation of P_n' at the converged node
                p0 = 1.0; p1 = z;
                for (int k = 1; k < n; ++k) {
                    const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                    p0 = p1;
                    p1 = p2;
                }
                if (n == 1) { p1 = z; p0 = 1.0; }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        // nodes ascending: x[i] = -z, x[n-1-i] = z
        x[i] = -z;
        x[n - 1 - i] = z;
        const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Product set: polar cosine xi = (1 + x)/2 on (0,1) with weight w_GL/2 (upper
// hemisphere), azimuths (2k-1) pi / n_azim; ordinate q = p * n_azim + (k-1);
// mu = sqrt(1-xi^2) cos, eta = sqrt(1-xi^2) sin, weight 4 pi om_p / n_azim.
void build_quadrature(int n_polar, int n_azim, std::vector<double>& mu, std::vector<double>& eta,
                      std::vector<double>& w) {
    std::vector<double> x, wg;
    gauss_legendre(n_polar, x, wg);
    const int nq = n_polar * n_azim;
    mu.resize(nq);
    eta.resize(nq);
    w.resize(nq);
    for (int p = 0; p < n_polar; ++p) {
        const double xi = 0.5 * (1.0 + x[p]);
        const double om = 0.5 * wg[p];
        const double s = std::sqrt(1.0 - xi * xi);
        for (int k = 0; k < n_azim; ++k) {
            const double ph = (2.0 * (k + 1) - 1.0) * kPi / n_azim;
            const int q = p * n_azim + k;
            mu[q] = s * std::cos(ph);
            eta[q] = s * std::sin(ph);
            w[q] = 4.0 * kPi * om / n_azim;
        }
    }
}

// Weighted classical Gram-Schmidt with one reorthogonalisation on an n x r
// column-major array Q (columns already accepted: 0..k-1).  Returns the norm of
// the residual and leaves it (normalised when nonzero) in v.
static double cgs2_residual(const std::vector<double>& Q, int n, int k, const std::vector<double>& wt,
                            std::vector<double>& v) {
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<double> h(k, 0.0);
        for (int j = 0; j < k; ++j) {
            const double* qj = &Q[(size_t)j * n];
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += qj[i] * wt[i] * v[i];
            h[j] = s;
        }
        for (int j = 0; j < k; ++j) {
            const double* qj = &Q[(size_t)j * n];
            for (int i = 0; i < n; ++i) v[i] -= h[j] * qj[i];
        }
    }
    double nn = 0.0;
    for (int i = 0; i < n; ++i) nn += wt[i] * v[i] * v[i];
    return std::sqrt(nn);
}

// Angular factor of the initial state: W_1 = 1/sqrt(4 pi), then graded
// monomials 1, mu, eta, mu^2, mu eta, eta^2, ... orthonormalised (CGS2) in the
// quadrature inner product, skipping those whose residual is below 1e-10 of
// their own norm.  Output column-major [r][nq].
static void angular_basis(const std::vector<double>& mu, const std::vector<double>& eta,
                          const std::vector<double>& w, int r, std::vector<double>& W) {
    const int nq = (int)mu.size();
    W.assign((size_t)r * nq, 0.0);
    double wsum = 0.0;
    for (double v : w) wsum += v;
    for (int q = 0; q < nq; ++q) W[q] = 1.0 / std::sqrt(wsum);
    int k = 1;
    for (int deg = 0; k < r && deg < 4 * nq; ++deg) {
        for (int ax = deg; ax >= 0 && k < r; --ax) {
            std::vector<double> v(nq);
            double own = 0.0;
            for (int q = 0; q < nq; ++q) {
                v[q] = std::pow(mu[q], ax) * std::pow(eta[q], deg - ax);
                own += w[q] * v[q] * v[q];
            }
            own = std::sqrt(own);
            const double res = cgs2_residual(W, nq, k, w, v);
            if (res > 1e-10 * own) {
                for (int q = 0; q < nq; ++q) W[(size_t)k * nq + q] = v[q] / res;
                ++k;
            }
        }
    }
    if (k < r) throw std::runtime_error("angular completion ran out of monomials");
}

void build_initial_factors(const ProblemHost& P, const std::vector<double>& mu, const std::vector<double>& eta,
                           const std::vector<double>& w, std::vector<double>& X, std::vector<double>& S,
                           std::vector<double>& W) {
    const int n = P.nx * P.ny, r = P.rank;
    const double area = P.hx * P.hy;
    angular_basis(mu, eta, w, r, W);
    double wsum = 0.0;
    for (double v : w) wsum += v;
    // x0 = B(T_init) / ||B||_X (or the constant when B == 0)
    std::vector<double> b(n);
    double nb = 0.0;
    for (int e = 0; e < n; ++e) {
        const double t = P.T_init[e];
        b[e] = P.a * P.c * t * t * t * t / (4.0 * kPi);
        nb += area * b[e] * b[e];
    }
    nb = std::sqrt(nb);
    std::vector<double> x0(n);
    for (int e = 0; e < n; ++e) x0[e] = (nb > 0.0) ? b[e] / nb : 1.0 / std::sqrt(area * n);
    // Columns 2..r: a Householder completion in the area-weighted inner product.
    // With u = x0 - e_1 (e_1 = cell 0 / sqrt(area)), H = I - 2 u u^T A / (u^T A u)
    // maps e_1 to x0, so H e_k (k >= 2) are orthonormal and orthogonal to x0.
    // These columns only meet zero entries of S, so they do not affect the plain step (instances
    // with the augmented basis, whose Galerkin space takes all of span X, replace them on the device).
    X.assign((size_t)r * n, 0.0);
    for (int e = 0; e < n; ++e) X[e] = x0[e];
    if (r > 1) {
        std::vector<double> u(x0);
        const double e1 = 1.0 / std::sqrt(area);
        u[0] -= e1;
        double uu = 0.0;
        for (int e = 0; e < n; ++e) uu += area * u[e] * u[e];
        for (int k = 1; k < r; ++k) {
            double* col = &X[(size_t)k * n];
            const int cell = k;   // e_k = cell k / sqrt(area)
            col[cell] = e1;
            if (uu > 0.0) {
                const double f = 2.0 * area * u[cell] * e1 / uu;
                for (int e = 0; e < n; ++e) col[e] -= f * u[e];
            }
        }
    }
    S.assign((size_t)r * r, 0.0);
    S[0] = nb * std::sqrt(wsum);
}

}  // namespace dlr
