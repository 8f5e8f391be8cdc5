"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C sweep (oracle/sweep.c) and the library's host-side set-up
(paper_2601_18705_amd/csrc/host_setup.cpp: Gauss-Legendre nodes, the product
quadrature, the initial factors with their completions) are compiled with
-fsanitize=address,undefined into small drivers that exercise them on tiny and
ragged shapes and check results with closed forms; any out-of-bounds access,
use of freed memory or undefined behaviour aborts the driver.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

SWEEP_DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
void oracle_sweep(int nx, int ny, double hx, double hy, int nd, const double *mu, const double *eta,
                  const double *sigt, const double *rhs, const double *inx, const double *iny, double *psi);
/* Equilibrium: with rhs = s sigma_t everywhere and inflow s on every inflow face, psi = s exactly
   (each cell's balance is satisfied by the constant); every orientation and shape. */
int main(void) {
    const int shapes[][2] = {{1, 1}, {1, 7}, {7, 1}, {5, 3}, {64, 2}, {65, 9}, {130, 4}};
    const double mus[4] = {0.3, -0.7, 0.45, -0.2}, etas[4] = {0.6, 0.25, -0.5, -0.9};
    for (unsigned k = 0; k < sizeof(shapes) / sizeof(shapes[0]); ++k) {
        const int nx = shapes[k][0], ny = shapes[k][1], nd = 4;
        const long n = (long)nx * ny;
        double *sig = malloc(n * sizeof(double)), *rhs = malloc(nd * n * sizeof(double));
        double *inx = malloc(nd * ny * sizeof(double)), *iny = malloc(nd * nx * sizeof(double));
        double *psi = malloc(nd * n * sizeof(double));
        const double s = 0.75;
        for (long e = 0; e < n; ++e) sig[e] = 1.0 + 0.5 * (double)(e % 7);
        for (int d = 0; d < nd; ++d) {
            for (long e = 0; e < n; ++e) rhs[d * n + e] = s * sig[e];
            for (int j = 0; j < ny; ++j) inx[d * ny + j] = s;
            for (int i = 0; i < nx; ++i) iny[d * nx + i] = s;
        }
        oracle_sweep(nx, ny, 1.0 / nx, 1.0 / ny, nd, mus, etas, sig, rhs, inx, iny, psi);
        for (long e = 0; e < nd * n; ++e)
            if (fabs(psi[e] - s) > 1e-14) { printf("mismatch shape %d e %ld: %g\n", k, e, psi[e]); return 1; }
        free(sig); free(rhs); free(inx); free(iny); free(psi);
    }
    printf("sweep ok\n");
    return 0;
}
"""

SETUP_DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <vector>
#include "host_setup.h"
int main() {
    const double pi = 3.14159265358979323846;
    for (int n = 1; n <= 64; ++n) {            // Gauss-Legendre on [-1, 1]: weights sum to 2, x^2 integrates to 2/3
        std::vector<double> x, w;
        dlr::gauss_legendre(n, x, w);
        double s0 = 0, s2 = 0;
        for (int i = 0; i < n; ++i) { s0 += w[i]; s2 += w[i] * x[i] * x[i]; }
        if (std::fabs(s0 - 2.0) > 1e-13 || (n >= 2 && std::fabs(s2 - 2.0 / 3.0) > 1e-13)) { std::printf("GL %d\n", n); return 1; }
    }
    const int quads[][2] = {{1, 4}, {2, 8}, {3, 4}, {8, 8}, {4, 12}};
    for (auto& q : quads) {
        std::vector<double> mu, eta, w;
        dlr::build_quadrature(q[0], q[1], mu, eta, w);
        double s = 0;
        for (double v : w) s += v;
        if ((int)w.size() != q[0] * q[1] || std::fabs(s - 4 * pi) > 1e-12) { std::printf("quad\n"); return 1; }
        const int grids[][2] = {{1, 1}, {3, 2}, {7, 5}, {16, 9}};
        for (auto& g : grids) {
            const int nq = q[0] * q[1], ncell = g[0] * g[1];
            const int rmax = nq < ncell ? nq : ncell;
            for (int r = 1; r <= rmax && r <= 12; r += 3) {
                std::vector<double> T(ncell, 0.1), X, S, W;
                dlr::ProblemHost P{g[0], g[1], r, 1.0 / g[0], 1.0 / g[1], 1.0, 1.0, T.data()};
                dlr::build_initial_factors(P, mu, eta, w, X, S, W);
                const double area = P.hx * P.hy;
                for (int a = 0; a < r; ++a)          // X^T (area) X = I and W^T diag(w) W = I
                    for (int b = 0; b < r; ++b) {
                        double gx = 0, gw = 0;
                        for (int e = 0; e < ncell; ++e) gx += area * X[(size_t)a * ncell + e] * X[(size_t)b * ncell + e];
                        for (int k = 0; k < nq; ++k) gw += w[k] * W[(size_t)a * nq + k] * W[(size_t)b * nq + k];
                        const double want = a == b ? 1.0 : 0.0;
                        if (std::fabs(gx - want) > 1e-10 || std::fabs(gw - want) > 1e-10) {
                            std::printf("orthonormality %d %d r %d grid %dx%d\n", a, b, r, g[0], g[1]);
                            return 1;
                        }
                    }
            }
        }
    }
    std::printf("setup ok\n");
    return 0;
}
"""


def _run(tmp_path, name, src, compiler, extra, lang_ext):
    drv = tmp_path / f"{name}_driver.{lang_ext}"
    drv.write_text(src)
    exe = tmp_path / name
    cmd = [compiler, *SAN, str(drv), *extra, "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr.lower() or "sanitizer" in r.stderr.lower()):
        pytest.skip("the host compiler has no sanitizer runtime here: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_sweep_under_sanitizers(tmp_path):
    out = _run(tmp_path, "sweep", SWEEP_DRIVER, "gcc", [os.path.join(ROOT, "oracle", "sweep.c")], "c")
    assert "sweep ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_setup_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2601_18705_amd", "csrc")
    out = _run(tmp_path, "setup", SETUP_DRIVER, "g++",
               ["-std=c++17", "-I", csrc, os.path.join(csrc, "host_setup.cpp")], "cpp")
    assert "setup ok" in out
