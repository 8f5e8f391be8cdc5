// Host-side set-up helpers (ordinates, initial factors).
#pragma once

#include <vector>

namespace dlr {

struct ProblemHost {
    int nx, ny, rank;
    double hx, hy, a, c;
    const double* T_init;
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void build_quadrature(int n_polar, int n_azim, std::vector<double>& mu, std::vector<double>& eta,
                      std::vector<double>& w);
// X [r][n] column-major, S [r][r] row-major, W [r][nq] column-major
void build_initial_factors(const ProblemHost& P, const std::vector<double>& mu, const std::vector<double>& eta,
                           const std::vector<double>& w, std::vector<double>& X, std::vector<double>& S,
                           std::vector<double>& W);

}  // namespace dlr
