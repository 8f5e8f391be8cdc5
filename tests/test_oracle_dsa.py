"""Pins of the oracle's diffusion synthetic acceleration (the DSA of the SN-like DLR
source iteration, Sec. 4 "Diffusion Synthetic Acceleration" and its appendix derivation),
for degree-0 elements.

* The face operators F_x, F_y (the part of the face matrix linear in Omega) are checked
  against a brute-force evaluation of the bilinear form sum_faces -h n_j [[v]] {{u}} on
  unit vectors, independent of the sparse assembly.
* The diffusion part (1/3) sum_j F_j^T M_t^{-1} F_j acts on a linear field as zero and on a
  quadratic field as -(2 area / (3 sigma_t)) in the interior: the consistent diffusion
  operator -div (1 / (3 sigma_t)) grad, exactly, on the wide stencil.
* The DSA matrix is symmetric positive definite; the penalty vanishes on constants in the
  interior and its coefficient for full quadrature weights is sum_q w_q |mu_q| (close to 2 pi).
* Accelerated source iteration reaches the unaccelerated fixed point, with far fewer
  iterations on an optically thick checkerboard (sigma = 10^4), for DLR and for plain SN.
* The exact sparse solve equals a dense solve of the same system on a 4 x 4 grid.
"""
import numpy as np
import pytest

from oracle import dlr_oracle as O
from synth import problems


def small_grid(nx=6, ny=5):
    return O.Grid(nx, ny, 0.0, 1.2, 0.0, 0.7)


def brute_face_form(grid, axis, v, u):
    """sum over faces of -h n_j [[v]] {{u}} with exterior values 0 (normal along +axis)."""
    V = v.reshape(grid.ny, grid.nx)
    U = u.reshape(grid.ny, grid.nx)
    total = 0.0
    if axis == 0:
        for j in range(grid.ny):
            for a in range(grid.nx + 1):
                vm = V[j, a - 1] if a > 0 else 0.0
                vp = V[j, a] if a < grid.nx else 0.0
                um = U[j, a - 1] if a > 0 else 0.0
                up = U[j, a] if a < grid.nx else 0.0
                total += -grid.hy * (vm - vp) * 0.5 * (um + up)
    else:
        for b in range(grid.ny + 1):
            for i in range(grid.nx):
                vm = V[b - 1, i] if b > 0 else 0.0
                vp = V[b, i] if b < grid.ny else 0.0
                um = U[b - 1, i] if b > 0 else 0.0
                up = U[b, i] if b < grid.ny else 0.0
                total += -grid.hx * (vm - vp) * 0.5 * (um + up)
    return total


@pytest.mark.parametrize("axis", [0, 1])
def test_face_operator_matches_bilinear_form(axis):
    g = small_grid()
    F = O.dsa_face_operators(g)[axis].toarray()
    n = g.ncell
    rng = np.random.default_rng(axis)
    for _ in range(6):
        v, u = rng.standard_normal(n), rng.standard_normal(n)
        assert abs(v @ F @ u - brute_face_form(g, axis, v, u)) < 1e-12


def test_diffusion_part_is_consistent_on_linear_and_quadratic_fields():
    g = O.Grid(12, 10, 0.0, 1.0, 0.0, 0.5)
    sig = 3.7
    Fx, Fy = O.dsa_face_operators(g)
    Dd = (Fx.T @ Fx + Fy.T @ Fy).toarray() / (3.0 * sig * g.area)
    x = (np.arange(g.nx) + 0.5) * g.hx
    y = (np.arange(g.ny) + 0.5) * g.hy
    X, Y = np.meshgrid(x, y)
    interior = np.zeros((g.ny, g.nx), bool)
    interior[2:-2, 2:-2] = True
    interior = interior.ravel()
    lin = (2.0 * X - 3.0 * Y + 1.0).ravel()
    assert np.max(np.abs((Dd @ lin)[interior])) < 1e-12
    quad = (X ** 2 + 0.5 * Y ** 2).ravel()
    want = -g.area * (2.0 + 1.0) / (3.0 * sig)   # -(1/(3 sigma)) (d2/dx2 + d2/dy2) times the cell area
    assert np.max(np.abs((Dd @ quad)[interior] - want)) < 1e-12


def test_dsa_matrix_is_spd_and_penalty_vanishes_on_interior_constants():
    g = small_grid()
    rng = np.random.default_rng(3)
    sig_t = rng.uniform(1.0, 50.0, g.ncell)
    sig_s = sig_t * rng.uniform(0.0, 0.99, g.ncell)
    D = O.dsa_matrix(g, sig_t, sig_s, 1.3, 0.9).toarray()
    assert np.max(np.abs(D - D.T)) < 1e-14 * np.max(np.abs(D))
    assert np.min(np.linalg.eigvalsh(D)) > 0.0
    P = O.dsa_penalty(g, 1.3, 0.9).toarray()
    one = np.ones(g.ncell)
    inner = np.zeros((g.ny, g.nx), bool)
    inner[1:-1, 1:-1] = True
    assert np.max(np.abs((P @ one)[inner.ravel()])) < 1e-15


def test_penalty_coefficient_for_full_quadrature():
    quad = O.quadrature(32, 64)
    kx, ky = O.dsa_kappas(quad.w, quad.mu, quad.eta)
    assert abs(kx - np.sum(quad.w * np.abs(quad.mu))) < 1e-15
    assert abs(kx - 2 * np.pi) < 5e-3 and abs(ky - 2 * np.pi) < 5e-3   # int over the sphere of |Omega . n| = 2 pi


def test_exact_solve_equals_dense_solve_on_4x4():
    g = O.Grid(4, 4, 0.0, 1.0, 0.0, 1.0)
    rng = np.random.default_rng(5)
    sig_t = rng.uniform(1.0, 1e3, g.ncell)
    sig_s = sig_t * rng.uniform(0.5, 0.999, g.ncell)
    lin = O.Linearised(D=np.ones(g.ncell), sigma_s=sig_s, q=np.zeros(g.ncell), sigma_t=sig_t,
                       emis0=np.zeros(g.ncell))
    half, old = rng.uniform(0, 1, g.ncell), rng.uniform(0, 1, g.ncell)
    got = O.dsa_correct(g, lin, (2.1, 1.7), half, old)
    D = O.dsa_matrix(g, sig_t, sig_s, 2.1, 1.7).toarray()
    want = half + np.linalg.solve(D, g.area * sig_s * (half - old))
    assert np.max(np.abs(got - want)) < 1e-13 * np.max(np.abs(want))


def thick_checkerboard(thick, n=28):
    p = problems.checkerboard(n=n, n_polar=4, n_azim=8, rank=8, nsteps=2)
    p["sigma_a"] = problems.checkerboard_sigma(p, thick=thick, thin=1.0)
    p["T_init"] = np.full(p["nx"] * p["ny"], 1.0)
    p["si_tol"] = 1e-13
    return p


def test_dsa_dlr_same_fixed_point_far_fewer_iterations():
    p = thick_checkerboard(1e4)
    _, plain = O.run_dlr(dict(p, dsa=0), nsteps=2)
    _, acc = O.run_dlr(dict(p, dsa=1), nsteps=2)
    for a, b in zip(acc, plain):
        assert np.max(np.abs(a["T"] - b["T"])) <= 1e-11 * np.max(np.abs(b["T"]))
        assert np.linalg.norm(a["E_r"] - b["E_r"]) <= 1e-10 * np.linalg.norm(b["E_r"])
    assert max(h["si_iters"] for h in plain) > 300
    assert max(h["si_iters"] for h in acc) <= 6


def test_dsa_plain_sn_same_fixed_point_far_fewer_iterations():
    p = thick_checkerboard(1e4, n=21)
    _, plain = O.run_sn(dict(p, dsa=0), nsteps=1)
    _, acc = O.run_sn(dict(p, dsa=1), nsteps=1)
    assert np.max(np.abs(acc[0]["T"] - plain[0]["T"])) <= 1e-11 * np.max(np.abs(plain[0]["T"]))
    assert plain[0]["si_iters"] > 300 and acc[0]["si_iters"] <= 6
