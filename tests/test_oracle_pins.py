"""Pins of the FP64 oracle against what the mathematics fixes.

The paper prints no worked numerical example, so every pin is a closed form,
an invariant, a reduction to a textbook or library routine, or a brute-force
dense solve on a tiny grid.  Each is chosen so that a plausible slip in the
oracle (dropped term, wrong sign, wrong upwind neighbour, transposed operand)
fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import dlr_oracle as O
from synth import problems

FOUR_PI = 4.0 * math.pi


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


# ============================================================================ quadrature

@pytest.mark.parametrize("npol,naz", [(2, 4), (8, 8), (16, 32), (5, 12)])
def test_quadrature_moments(npol, naz):
    q = O.quadrature(npol, naz)
    assert abs(q.w.sum() - FOUR_PI) < 1e-13
    assert abs(q.w @ q.mu) < 1e-14 and abs(q.w @ q.eta) < 1e-14
    assert abs(q.w @ (q.mu * q.eta)) < 1e-14
    # int mu^2 = int eta^2 = int xi^2 = 4 pi / 3 over the sphere (xy symmetry doubles the hemisphere)
    assert abs(q.w @ q.mu ** 2 - FOUR_PI / 3) < 1e-13
    assert abs(q.w @ q.eta ** 2 - FOUR_PI / 3) < 1e-13
    assert abs(q.w @ q.xi ** 2 - FOUR_PI / 3) < 1e-13
    # int mu^4 = 4 pi / 5 needs (1 - xi^2)^2 (Gauss, n >= 3) and cos^4 (n_azim > 4) exact
    if npol >= 3 and naz > 4:
        assert abs(q.w @ q.mu ** 4 - FOUR_PI / 5) < 1e-12
    assert np.all(np.abs(q.mu) > 1e-3) and np.all(np.abs(q.eta) > 1e-3)
    # mirror maps are involutions onto the exact mirrored ordinate with equal weight
    for m, sx, sy in ((q.refl_x, -1, 1), (q.refl_y, 1, -1)):
        assert np.all(m[m] == np.arange(q.n))
        assert np.allclose(q.mu[m], sx * q.mu, atol=1e-15) and np.allclose(q.eta[m], sy * q.eta, atol=1e-15)
        assert np.allclose(q.w[m], q.w, rtol=0, atol=1e-15)


def test_gauss_legendre_polar_exactness():
    """n-point Gauss-Legendre on (0,1) integrates xi^k exactly for k <= 2n - 1;
    with the unit-sum weights, sum_p om_p xi_p^k = 1/(k+1)."""
    for n in (1, 2, 3, 8, 16, 32):
        q = O.quadrature(n, 4)
        xi = q.xi[::4]
        om = q.w[::4] * 4 / FOUR_PI
        for k in range(2 * n):
            assert abs(om @ xi ** k - 1.0 / (k + 1)) < 1e-13
    # the 2-point rule in closed form: nodes (1 -+ 1/sqrt 3)/2, equal weights
    q = O.quadrature(2, 4)
    assert np.allclose(np.sort(q.xi[::4]), [(1 - 1 / math.sqrt(3)) / 2, (1 + 1 / math.sqrt(3)) / 2], atol=1e-15)


# ============================================================================ linearisation

def _rand_cells(rng, n):
    return dict(T0=rng.uniform(0.05, 2.0, n), sig=rng.uniform(0.1, 50.0, n), rcv=rng.uniform(0.1, 3.0, n),
                phi=rng.uniform(0.0, 10.0, n))


def test_temperature_update_is_one_newton_step():
    """T = T0 - F(T0)/F'(T0) for F(T) = rho c_v (T - T0) - dt sigma (phi - 4 pi B(T)),
    with F' taken by a central finite difference of F (independent of B')."""
    rng = np.random.default_rng(1)
    n = 64
    c = _rand_cells(rng, n)
    p = dict(sigma_a=c["sig"], rho_cv=c["rcv"], q_ext=np.zeros(n), dt=0.013, a=0.7, c=1.9)
    lin = O.linearise(p, c["T0"])
    T = O.temperature_update(p, c["T0"], lin, c["phi"])

    def F(Tv):
        return p["rho_cv"] * (Tv - c["T0"]) - p["dt"] * p["sigma_a"] * (c["phi"] - p["a"] * p["c"] * Tv ** 4)

    h = 1e-6 * c["T0"]
    dF = (F(c["T0"] + h) - F(c["T0"] - h)) / (2 * h)
    newton = c["T0"] - F(c["T0"]) / dF
    assert np.max(np.abs(T - newton) / np.abs(newton)) < 1e-8


def test_effective_scattering_and_source_reproduce_linearised_emission():
    """sigma B(T_lin) to first order equals sigma_s phi/(4 pi) + q (q_ext = 0):
    sigma (B(T0) + B'(T0)(T - T0)) with B' by finite differences of a c T^4/(4 pi)."""
    rng = np.random.default_rng(2)
    n = 64
    c = _rand_cells(rng, n)
    p = dict(sigma_a=c["sig"], rho_cv=c["rcv"], q_ext=np.zeros(n), dt=0.02, a=1.3, c=0.8)
    lin = O.linearise(p, c["T0"])
    T = O.temperature_update(p, c["T0"], lin, c["phi"])

    def B(Tv):
        return p["a"] * p["c"] * Tv ** 4 / FOUR_PI

    h = 1e-6 * c["T0"]
    dB = (B(c["T0"] + h) - B(c["T0"] - h)) / (2 * h)
    emis = p["sigma_a"] * (B(c["T0"]) + dB * (T - c["T0"]))
    model = lin.sigma_s * c["phi"] / FOUR_PI + lin.q
    assert np.max(np.abs(emis - model) / np.abs(model)) < 1e-8
    # external source enters the transport source as q_ext / (4 pi)
    p2 = dict(p, q_ext=np.full(n, 3.0))
    assert np.allclose(O.linearise(p2, c["T0"]).q - lin.q, 3.0 / FOUR_PI, rtol=1e-14)
    # sigma_t = sigma + 1/(c dt)
    assert np.allclose(lin.sigma_t, p["sigma_a"] + 1.0 / (p["c"] * p["dt"]), rtol=1e-15)


def test_linearisation_limits_and_equilibrium():
    rng = np.random.default_rng(3)
    n = 16
    c = _rand_cells(rng, n)
    p = dict(sigma_a=c["sig"], rho_cv=c["rcv"], q_ext=np.zeros(n), dt=1e-14, a=1.0, c=1.0)
    lin = O.linearise(p, c["T0"])
    assert np.max(lin.sigma_s / c["sig"]) < 1e-11          # dt -> 0: no pseudo-scattering
    assert np.allclose(lin.q, c["sig"] * c["T0"] ** 4 / FOUR_PI, rtol=1e-10)   # q -> sigma B
    p["dt"] = 0.5
    lin = O.linearise(p, c["T0"])
    T = O.temperature_update(p, c["T0"], lin, c["T0"] ** 4)   # phi = a c T0^4: equilibrium is a fixed point
    assert np.allclose(T, c["T0"], rtol=1e-15, atol=0)


# ============================================================================ (a) infinite homogeneous medium

def _infinite_medium(nx=3, npol=2, naz=4, rank=None, dt=0.01, nsteps=1, Tm=0.5, Tr=1.0, sigma=1.0, C=1.0):
    p = problems.base_problem(nx, nx, (0, 1, 0, 1), npol, naz, rank or npol * naz, dt, nsteps=nsteps)
    n = nx * nx
    p["sigma_a"] = np.full(n, sigma)
    p["rho_cv"] = np.full(n, C)
    p["bc"] = [O.BC_REFLECT] * 4
    p["T_init"] = np.full(n, Tr)          # radiation temperature of the initial field
    return p, np.full(n, Tm)


def _closed_form_recurrence(T, phi, sigma, C, dt, a=1.0, c=1.0, nsteps=1):
    """Uniform isotropic state: streaming vanishes and each step reduces to
    phi' (1/(c dt) + f sigma) = phi/(c dt) + f sigma a c T^4,
    T' = T + dt sigma (phi' - a c T^4)/D, f = C/D, D = C + 4 a c dt sigma T^3."""
    out = []
    for _ in range(nsteps):
        D = C + 4 * a * c * dt * sigma * T ** 3
        f = C / D
        phi = (phi / (c * dt) + f * sigma * a * c * T ** 4) / (1 / (c * dt) + f * sigma)
        T = T + dt * sigma * (phi - a * c * T ** 4) / D
        out.append((T, phi))
    return out


def test_infinite_medium_sn_matches_closed_form():
    p, Tm = _infinite_medium(nsteps=6)
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    st = O.sn_initial_state(p, quad)
    st.T = Tm.copy()
    ref = _closed_form_recurrence(0.5, 1.0, 1.0, 1.0, p["dt"], nsteps=6)
    for n in range(6):
        st, _ = O.sn_step(p, quad, st)
        assert np.max(np.abs(st.T / ref[n][0] - 1)) < 1e-13
        assert np.max(np.abs(st.phi / ref[n][1] - 1)) < 1e-13


@pytest.mark.parametrize("rank", [1, 2, 4, 8])
def test_infinite_medium_dlr_matches_closed_form_every_rank(rank):
    p, Tm = _infinite_medium(rank=rank, nsteps=4)
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    st = O.dlr_initial_state(p, quad)
    st.T = Tm.copy()
    ref = _closed_form_recurrence(0.5, 1.0, 1.0, 1.0, p["dt"], nsteps=4)
    for n in range(4):
        st, stats = O.dlr_step(p, quad, st)
        assert np.max(np.abs(st.T / ref[n][0] - 1)) < 1e-13
        assert np.max(np.abs(stats["phi"] / ref[n][1] - 1)) < 1e-13


def test_infinite_medium_relaxes_to_energy_equilibrium():
    """The limit T_eq solves C T + a T^4 = E (E = C T0 + phi0 / c conserved)."""
    p, Tm = _infinite_medium(nsteps=1, dt=0.05)
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    st = O.sn_initial_state(p, quad)
    st.T = Tm.copy()
    E = 1.0 * 0.5 + 1.0
    for _ in range(400):
        st, _ = O.sn_step(p, quad, st)
    Teq = scipy.optimize.brentq(lambda T: T + T ** 4 - E, 0.0, 2.0, xtol=1e-15)
    assert abs(st.T[0] - Teq) < 1e-12 and abs(st.phi[0] - Teq ** 4) < 1e-11


def test_infinite_medium_first_order_in_time():
    """Backward Euler with the Newton-linearised emission converges at first
    order to the ODE (1/c) phi' = sigma (a c T^4 - phi), C T' = sigma (phi - a c T^4)."""
    tend = 0.4

    def rhs(t, y):
        T, phi = y
        return [(phi - T ** 4), (T ** 4 - phi)]

    sol = scipy.integrate.solve_ivp(rhs, (0, tend), [0.5, 1.0], method="Radau", rtol=1e-12, atol=1e-14)
    Tex = sol.y[0, -1]
    errs = []
    for dt in (0.02, 0.01, 0.005):
        nst = int(round(tend / dt))
        p, Tm = _infinite_medium(nx=1, npol=1, naz=4, dt=dt, nsteps=nst)
        quad = O.quadrature(1, 4)
        st = O.sn_initial_state(p, quad)
        st.T = Tm.copy()
        for _ in range(nst):
            st, _ = O.sn_step(p, quad, st)
        errs.append(abs(st.T[0] - Tex))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(0.9 < s < 1.1 for s in slopes), slopes


# ============================================================================ (b) pure absorber

def test_pure_absorber_exact_discrete_attenuation():
    """T = 0: no emission, no pseudo-scattering.  One direction, left inflow psi_b,
    bottom inflow equal to the 1-D profile: psi_ij = psi_b (1 + sigma_t h/|mu|)^-(i+1)."""
    nx, ny = 24, 9
    grid = O.Grid(nx, ny, 0.0, 2.0, 0.0, 1.0)
    mu, eta = np.array([0.37]), np.array([0.52])
    sig = 3.0
    dt = 1e12
    sigt = np.full(grid.ncell, sig + 1.0 / dt)
    psib = 0.8
    g = 1.0 / (1.0 + sigt[0] * grid.hx / mu[0])
    prof = psib * g ** (np.arange(nx) + 1)
    psi = O.sweep(grid, mu, eta, sigt, np.zeros((1, grid.ncell)), np.full((1, ny), psib), prof[None, :])
    exact = np.tile(prof, ny)
    assert np.max(np.abs(psi[0] / exact - 1)) < 1e-14
    # mirrored direction: inflow from the right / top gives the mirrored profile
    psi2 = O.sweep(grid, -mu, -eta, sigt, np.zeros((1, grid.ncell)), np.full((1, ny), psib), prof[::-1][None, :])
    assert np.max(np.abs(psi2[0] / np.tile(prof[::-1], ny) - 1)) < 1e-14


def test_pure_absorber_converges_to_exponential_first_order():
    """psi -> psi_b exp(-sigma x / mu) at first order in h (cell-average of the exact ray)."""
    errs = []
    sig, mu0, psib = 2.0, 0.6, 1.0
    for nx in (128, 256, 512, 1024):
        grid = O.Grid(nx, 2, 0.0, 1.0, 0.0, 1.0)
        g = 1.0 / (1.0 + sig * grid.hx / mu0)
        prof = psib * g ** (np.arange(nx) + 1)
        psi = O.sweep(grid, np.array([mu0]), np.array([0.3]), np.full(grid.ncell, sig),
                      np.zeros((1, grid.ncell)), np.full((1, 2), psib), prof[None, :])
        xl = np.arange(nx) * grid.hx
        cell_avg = psib * mu0 / (sig * grid.hx) * (np.exp(-sig * xl / mu0) - np.exp(-sig * (xl + grid.hx) / mu0))
        errs.append(np.max(np.abs(psi[0, :nx] - cell_avg)))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(0.9 < s < 1.15 for s in slopes), slopes


# ============================================================================ (c) energy conservation

def _hetero(nx=5, ny=4, npol=2, naz=4, bc=None, seed=7, dt=0.02):
    rng = np.random.default_rng(seed)
    p = problems.base_problem(nx, ny, (0, 1.0, 0, 0.8), npol, naz, npol * naz, dt)
    n = nx * ny
    p["sigma_a"] = rng.uniform(0.5, 5.0, n)
    p["rho_cv"] = rng.uniform(0.5, 2.0, n)
    T = np.full(n, 0.1)
    T[rng.integers(0, n)] = 1.0
    p["T_init"] = T
    p["bc"] = bc or [O.BC_REFLECT] * 4
    return p


def test_energy_conserved_reflecting_sn_and_full_rank_dlr():
    p = _hetero()
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    sn = O.sn_initial_state(p, quad)
    dl = O.dlr_initial_state(p, quad)
    E0 = O.total_energy(p, grid, sn.T, sn.phi)
    for _ in range(5):
        sn, _ = O.sn_step(p, quad, sn)
        dl, stats = O.dlr_step(p, quad, dl)
        assert abs(O.total_energy(p, grid, sn.T, sn.phi) / E0 - 1) < 1e-12
        assert abs(O.total_energy(p, grid, dl.T, stats["phi"]) / E0 - 1) < 1e-12
    assert sn.T.max() < 0.99   # something actually moved


def _open_problem():
    p = _hetero(bc=[O.BC_INFLOW, O.BC_VACUUM, O.BC_INFLOW, O.BC_VACUUM])
    p["T_b"] = [1.0, 0.0, 0.5, 0.0]
    p["q_ext"] = np.linspace(0.0, 2.0, p["nx"] * p["ny"])
    return p


def test_energy_balance_with_inflow_vacuum_and_source():
    """E_new - E_old = dt (boundary inflow - outflow + int q_ext) for plain SN, with the
    oracle's boundary tally (inflow and outflow from the end-of-step intensity)."""
    p = _open_problem()
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    st = O.sn_initial_state(p, quad)
    for _ in range(3):
        E0 = O.total_energy(p, grid, st.T, st.phi)
        st, stats = O.sn_step(p, quad, st)
        E1 = O.total_energy(p, grid, st.T, st.phi)
        assert abs(stats["energy"] - E1) <= 1e-15 * E1
        assert stats["inflow"] > 0 and stats["outflow"] > 0
        dE = p["dt"] * (stats["inflow"] - stats["outflow"] + O.source_power(p, grid))
        assert abs((E1 - E0) - dE) < 1e-12 * E1


def test_energy_balance_full_rank_dlr_from_factors():
    """The same balance for full-rank DLR, the outflow evaluated from the new factors
    X S W^T on the wall cells; both flows equal plain SN's."""
    p = _open_problem()
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    dl = O.dlr_initial_state(p, quad)
    sn = O.sn_initial_state(p, quad)
    E0 = O.total_energy(p, grid, dl.T, O.mean_intensity(quad, dl))
    for _ in range(3):
        dl, stats = O.dlr_step(p, quad, dl)
        sn, sst = O.sn_step(p, quad, sn)
        E1 = stats["energy"]
        dE = p["dt"] * (stats["inflow"] - stats["outflow"] + O.source_power(p, grid))
        assert abs((E1 - E0) - dE) < 1e-11 * E1
        assert abs(stats["inflow"] - sst["inflow"]) < 1e-12 * sst["inflow"]
        assert abs(stats["outflow"] - sst["outflow"]) < 1e-10 * sst["outflow"]
        E0 = E1


def test_boundary_flows_single_side_closed_form():
    """One inflow side: the inflow is psi_b x side length x sum of w |mu| over the entering
    ordinates (half of sum_q w_q |mu_q| by the quadrature's mirror symmetry), and a field that
    is zero on every wall cell has no outflow; a uniform field psi = 1 leaves through each side
    at length x sum over exiting ordinates of w |Omega . n|."""
    p = _hetero(nx=6, ny=3, bc=[O.BC_VACUUM] * 4)
    p["bc"][O.SIDE_LEFT] = O.BC_INFLOW
    p["T_b"] = [0.7, 0, 0, 0]
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    psib = O.planck(0.7, p["a"], p["c"])
    zero = O.boundary_flows(p, grid, quad, lambda side: np.zeros((quad.n, O.side_cells(grid, side).size)))
    height = grid.y1 - grid.y0
    assert abs(zero[0] - psib * height * 0.5 * np.sum(quad.w * np.abs(quad.mu))) < 1e-14
    assert zero[1] == 0.0
    one = O.boundary_flows(p, grid, quad, lambda side: np.ones((quad.n, O.side_cells(grid, side).size)))
    width = grid.x1 - grid.x0
    expect = 2 * height * 0.5 * np.sum(quad.w * np.abs(quad.mu)) + 2 * width * 0.5 * np.sum(quad.w * np.abs(quad.eta))
    assert abs(one[1] - expect) < 1e-13 * expect


def test_reflecting_walls_have_no_net_flow():
    p = _hetero()
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    st = O.sn_initial_state(p, quad)
    for _ in range(2):
        st, stats = O.sn_step(p, quad, st)
        assert abs(stats["inflow"] - stats["outflow"]) < 1e-12 * stats["outflow"]


def test_deim_decision_edge():
    """The decision edge is the smallest distance of |R_q| / max |R| from the tie threshold."""
    W = np.array([[0.5], [1.0], [0.2], [0.999_999_5]])
    sel, margins, edge = O.deim(W, 1e-6, edges=True)
    assert sel[0] == 1 and abs(edge[0] - 0.5e-6) < 1e-15
    sel, margins, edge = O.deim(np.array([[0.5], [1.0], [0.2], [0.9]]), 1e-6, edges=True)
    assert abs(edge[0] - (1.0 - 1e-6 - 0.9)) < 1e-15 and abs(margins[0] - 0.1) < 1e-15


# ============================================================================ (d) full rank == plain SN

def test_full_rank_dlr_reproduces_plain_sn():
    p = problems.slab_beam(nx=32, n_polar=8, n_azim=8, rank=64, nsteps=10)
    quad = O.quadrature(8, 8)
    sn = O.sn_initial_state(p, quad)
    dl = O.dlr_initial_state(p, quad)
    for n in range(10):
        sn, _ = O.sn_step(p, quad, sn)
        dl, stats = O.dlr_step(p, quad, dl)
        assert sorted(stats["sel"].tolist()) == list(range(64))
        assert np.allclose(stats["cw"], quad.w[stats["sel"]], rtol=1e-12, atol=0)
        assert rel(stats["phi"], sn.phi) < 1e-11
        assert rel(dl.T, sn.T) < 1e-11


# ============================================================================ brute force on tiny grids

def _dense_sn_system(p, quad, grid, lin, fixed_rhs, weights, mu, eta):
    """Assemble the coupled degree-0 upwind system for all given directions
    (unknown psi[d, e]) with isotropic coupling sigma_s/(4 pi) sum_k weights_k psi_k."""
    nd, n = mu.size, grid.ncell
    M = np.zeros((nd * n, nd * n))
    b = fixed_rhs.reshape(-1).copy()
    a_, c_ = p["a"], p["c"]
    for d in range(nd):
        ax, ay = abs(mu[d]) / grid.hx, abs(eta[d]) / grid.hy
        for j in range(grid.ny):
            for i in range(grid.nx):
                e = j * grid.nx + i
                row = d * n + e
                M[row, row] += lin.sigma_t[e] + ax + ay
                iu = i - 1 if mu[d] > 0 else i + 1
                ju = j - 1 if eta[d] > 0 else j + 1
                if 0 <= iu < grid.nx:
                    M[row, d * n + j * grid.nx + iu] -= ax
                else:
                    side = O.SIDE_LEFT if mu[d] > 0 else O.SIDE_RIGHT
                    if p["bc"][side] == O.BC_INFLOW:
                        b[row] += ax * O.planck(p["T_b"][side], a_, c_)
                if 0 <= ju < grid.ny:
                    M[row, d * n + ju * grid.nx + i] -= ay
                else:
                    side = O.SIDE_BOTTOM if eta[d] > 0 else O.SIDE_TOP
                    if p["bc"][side] == O.BC_INFLOW:
                        b[row] += ay * O.planck(p["T_b"][side], a_, c_)
                for k in range(nd):
                    M[row, k * n + e] -= lin.sigma_s[e] / FOUR_PI * weights[k]
    return np.linalg.solve(M, b).reshape(nd, n)


def _warm_tiny(nx=4, ny=4, npol=2, naz=4, rank=None):
    p = problems.base_problem(nx, ny, (0, 1.0, 0, 1.0), npol, naz, rank or npol * naz, dt=0.5)
    rng = np.random.default_rng(11)
    n = nx * ny
    p["sigma_a"] = rng.uniform(1.0, 8.0, n)
    p["T_init"] = rng.uniform(0.5, 1.0, n)
    p["q_ext"] = rng.uniform(0.0, 1.0, n)
    p["bc"] = [O.BC_INFLOW, O.BC_VACUUM, O.BC_VACUUM, O.BC_INFLOW]
    p["T_b"] = [1.2, 0.0, 0.0, 0.7]
    return p


def test_sn_source_iteration_matches_dense_solve():
    p = _warm_tiny()
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    st = O.sn_initial_state(p, quad)
    st.psi = st.psi * np.linspace(0.5, 1.5, quad.n)[:, None]   # anisotropic previous solution
    lin = O.linearise(p, st.T)
    new, info = O.sn_step(p, quad, st)
    assert info["si_iters"] > 5   # scattering is strong enough to need iterations
    fixed = lin.q[None, :] + st.psi / (p["c"] * p["dt"])
    dense = _dense_sn_system(p, quad, grid, lin, fixed, quad.w, quad.mu, quad.eta)
    assert rel(new.psi, dense) < 1e-12


def test_collocation_source_iteration_matches_dense_solve():
    p = _warm_tiny(rank=3)
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    st = O.dlr_initial_state(p, quad)
    st, _ = O.dlr_step(p, quad, st)          # a non-trivial basis
    lin = O.linearise(p, st.T)
    _, stats = O.dlr_step(p, quad, st)
    sel = stats["sel"]
    fixed = lin.q[None, :] + stats["Psi0"] / (p["c"] * p["dt"])
    dense = _dense_sn_system(p, quad, grid, lin, fixed, stats["cw"], quad.mu[sel], quad.eta[sel])
    assert rel(stats["Psi"], dense) < 1e-12


def _apply_transport(p, grid, mu, eta, sigma_t, u):
    """(T_Omega + sigma_t) u for a cell field u, vacuum outside (stencil form)."""
    U = u.reshape(grid.ny, grid.nx)
    up_x = np.zeros_like(U)
    up_y = np.zeros_like(U)
    if mu > 0:
        up_x[:, 1:] = U[:, :-1]
    else:
        up_x[:, :-1] = U[:, 1:]
    if eta > 0:
        up_y[1:, :] = U[:-1, :]
    else:
        up_y[:-1, :] = U[1:, :]
    out = abs(mu) / grid.hx * (U - up_x) + abs(eta) / grid.hy * (U - up_y)
    return out.ravel() + sigma_t * u


def _galerkin_residual(p, grid, quad, X, L, lin, Lt0):
    """Largest scaled X-projection of the transport residual of psi_q = X L_q,
    applied by a stencil; zero when L solves the Galerkin system on span(X)."""
    A = grid.area
    phi_L = X @ (quad.w @ L)
    psi0 = X @ Lt0.T   # projection of the old solution; only its X-components enter
    worst = 0.0
    for qi in range(quad.n):
        mu, eta = quad.mu[qi], quad.eta[qi]
        u = X @ L[qi]
        res = _apply_transport(p, grid, mu, eta, lin.sigma_t, u) - lin.sigma_s * phi_L / FOUR_PI - lin.q \
            - psi0[:, qi] / (p["c"] * p["dt"])
        # inflow faces act as sources on the first upwind column/row
        for side, cosn, h in ((O.SIDE_LEFT if mu > 0 else O.SIDE_RIGHT, abs(mu), grid.hx),
                              (O.SIDE_BOTTOM if eta > 0 else O.SIDE_TOP, abs(eta), grid.hy)):
            if p["bc"][side] == O.BC_INFLOW:
                res = res - cosn / h * O.planck(p["T_b"][side], p["a"], p["c"]) * grid.side_mask(side)
        proj = A * X.T @ res
        scale = A * np.abs(X.T) @ (np.abs(lin.sigma_t * u) + np.abs(lin.q))
        worst = max(worst, float(np.max(np.abs(proj) / scale)))
    return worst


def test_l_step_is_galerkin_projection():
    """L from the L-step makes the residual of the transport equation, applied
    to psi_q = X L_q by a stencil, orthogonal to every X_i."""
    p = _warm_tiny(nx=5, ny=4, npol=2, naz=8, rank=5)
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    grid = O.grid_of(p)
    st = O.dlr_initial_state(p, quad)
    st, _ = O.dlr_step(p, quad, st)
    _, stats = O.dlr_step(p, quad, st)
    assert _galerkin_residual(p, grid, quad, stats["X_pre"], stats["L"], stats["lin"], stats["Lt0"]) < 1e-12


# ============================================================================ DEIM, QR, SVD

def _lu_pivot_rows(W):
    """Row pivots, in order, of LAPACK getrf (partial pivoting) on W."""
    lu, piv = scipy.linalg.lu_factor(W)
    perm = np.arange(W.shape[0])
    for k, pk in enumerate(piv):
        perm[[k, pk]] = perm[[pk, k]]
    return perm[:W.shape[1]]


@pytest.mark.parametrize("n,r,seed", [(64, 8, 0), (512, 16, 1), (300, 24, 2)])
def test_deim_equals_partial_pivoting_lu(n, r, seed):
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((n, r))
    sel, _ = O.deim(W, 1e-6)
    assert np.array_equal(sel, _lu_pivot_rows(W))


def test_deim_weights_integrate_span_exactly():
    quad = O.quadrature(4, 8)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((quad.n, 6))
    W, _ = O.cgs2(V, quad.w, O.angular_completion(quad))
    sel, _ = O.deim(W, 1e-6)
    cw = np.linalg.solve(W[sel].T, W.T @ quad.w)
    for _ in range(5):
        f = W @ rng.standard_normal(6)
        assert abs(cw @ f[sel] - quad.w @ f) < 1e-13 * np.abs(quad.w * f).sum()
    # the constant function is in span W for the initial basis: weights sum to 4 pi
    p = problems.slab_beam(nx=4, rank=8)
    st = O.dlr_initial_state(p, quad)
    s0, _ = O.deim(st.W, 1e-6)
    cw0 = np.linalg.solve(st.W[s0].T, st.W.T @ quad.w)
    assert abs(cw0.sum() - FOUR_PI) < 1e-13


def test_deim_tie_rule_prefers_smallest_index():
    W = np.zeros((6, 1))
    W[:, 0] = [0.1, 0.5, -0.5 * (1 - 1e-9), 0.3, 0.5, 0.2]
    sel, margins = O.deim(W, 1e-6)
    assert sel[0] == 1 and abs(margins[0] - 0.4) < 1e-12


def test_cgs2_matches_library_qr_and_orthonormality():
    rng = np.random.default_rng(9)
    n, r = 200, 12
    A = 0.37
    V = rng.standard_normal((n, r)) @ np.diag(10.0 ** rng.uniform(-8, 2, r))
    grid = O.Grid(20, 10, 0, 1, 0, 1)
    Q, R = O.cgs2(V, np.full(n, A), O.spatial_completion(grid))
    assert np.max(np.abs(A * Q.T @ Q - np.eye(r))) < 1e-13
    assert np.max(np.abs(Q @ R - V)) < 1e-13 * np.abs(V).max()
    Ql, Rl = np.linalg.qr(math.sqrt(A) * V)
    s = np.sign(np.diag(Rl))
    assert np.max(np.abs(Q - Ql * s / math.sqrt(A))) < 1e-9
    # V = Q R with Q = Ql / sqrt(A) means R = Rl (row signs fixed)
    assert np.allclose(R, (Rl.T * s).T, rtol=1e-10, atol=1e-12 * np.abs(R).max())


def test_cgs2_completes_rank_deficient_columns():
    grid = O.Grid(6, 5, 0, 1, 0, 1)
    n = grid.ncell
    rng = np.random.default_rng(3)
    v = rng.standard_normal(n)
    V = np.stack([v, 2 * v, np.zeros(n), rng.standard_normal(n)], axis=1)
    Q, R = O.cgs2(V, np.full(n, grid.area), O.spatial_completion(grid))
    assert np.max(np.abs(grid.area * Q.T @ Q - np.eye(4))) < 1e-13
    assert np.max(np.abs(Q @ R - V)) < 1e-12
    assert R[1, 1] == 0.0 and R[2, 2] == 0.0 and R[3, 3] > 0


def test_svd_rotation_keeps_psi_and_orders_singular_values():
    rng = np.random.default_rng(4)
    X = np.linalg.qr(rng.standard_normal((40, 6)))[0]
    W = np.linalg.qr(rng.standard_normal((30, 6)))[0]
    S = rng.standard_normal((6, 6))
    X2, S2, W2 = O.svd_rotate(X, S, W)
    assert np.max(np.abs(X @ S @ W.T - X2 @ S2 @ W2.T)) < 1e-13
    d = np.diag(S2)
    assert np.all(np.diff(d) <= 0) and np.all(d >= 0)
    assert np.max(np.abs(S2 - np.diag(d))) == 0.0
    assert np.max(np.abs(X2.T @ X2 - np.eye(6))) < 1e-13
    for k in range(6):   # sign convention on the angular factor
        col = np.linalg.lstsq(W, W2[:, k], rcond=None)[0]
        assert col[np.argmax(np.abs(col))] > 0


# ============================================================================ DG0 structure

def test_sn_positivity_and_mirror_symmetry():
    p = problems.slab_beam(nx=12, n_polar=2, n_azim=8, nsteps=2)
    n = p["nx"] * p["ny"]
    yc = np.repeat((np.arange(12) + 0.5) / 12, 12)
    p["sigma_a"] = 1.0 + 5.0 * (np.abs(yc - 0.5) < 0.2)     # mirror-symmetric in y
    quad = O.quadrature(2, 8)
    st = O.sn_initial_state(p, quad)
    for _ in range(2):
        st, _ = O.sn_step(p, quad, st)
    assert np.all(st.psi >= 0)
    f = st.psi.reshape(quad.n, 12, 12)
    mirrored = f[quad.refl_y][:, ::-1, :]
    assert np.max(np.abs(f - mirrored)) < 1e-14 * f.max()
    T = st.T.reshape(12, 12)
    assert np.max(np.abs(T - T[::-1])) < 1e-14


# ============================================================================ augmented basis (rank 2r -> r)

def _augmented(p):
    q = dict(p)
    q["augment"] = True
    return q


@pytest.mark.parametrize("rank", [1, 2, 4])
def test_augmented_infinite_medium_matches_closed_form(rank):
    """The uniform isotropic state has rank one, so the truncation loses nothing and
    the augmented step follows the same scalar recurrence as plain SN."""
    p, Tm = _infinite_medium(rank=rank, nsteps=4)
    p = _augmented(p)
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    st = O.dlr_initial_state(p, quad)
    st.T = Tm.copy()
    ref = _closed_form_recurrence(0.5, 1.0, 1.0, 1.0, p["dt"], nsteps=4)
    for n in range(4):
        st, stats = O.dlr_step(p, quad, st)
        assert st.X.shape[1] == rank and stats["X_gal"].shape[1] == 2 * rank
        assert np.max(np.abs(st.T / ref[n][0] - 1)) < 1e-13
        assert np.max(np.abs(stats["phi"] / ref[n][1] - 1)) < 1e-13


def _warm_augmented(rank=3, nsteps=2):
    p = _augmented(_warm_tiny(nx=5, ny=4, npol=2, naz=8, rank=rank))
    quad = O.quadrature(p["n_polar"], p["n_azim"])
    st = O.dlr_initial_state(p, quad)
    for _ in range(nsteps - 1):
        st, _ = O.dlr_step(p, quad, st)
    return p, quad, O.grid_of(p), st


def test_augmented_basis_holds_the_old_solution():
    """With X0 inside the Galerkin space, projecting the old intensity onto it is
    exact: X_gal Lt0^T = X0 S0 W0^T.  The plain basis does not have this property,
    which the second half checks so that the pin can tell the two apart."""
    p, quad, grid, st = _warm_augmented()
    old = st.X @ st.S @ st.W.T
    _, stats = O.dlr_step(p, quad, st)
    Xg = stats["X_gal"]
    assert np.max(np.abs(grid.area * Xg.T @ Xg - np.eye(Xg.shape[1]))) < 1e-13
    assert rel(Xg @ stats["Lt0"].T, old) < 1e-13
    q = dict(p)
    q["augment"] = False
    _, plain = O.dlr_step(q, quad, st)
    assert rel(plain["X_gal"] @ plain["Lt0"].T, old) > 1e-6


def test_augmented_l_step_is_galerkin_projection_on_2r_columns():
    p, quad, grid, st = _warm_augmented()
    _, stats = O.dlr_step(p, quad, st)
    assert stats["L"].shape == (quad.n, 2 * st.X.shape[1])
    assert _galerkin_residual(p, grid, quad, stats["X_gal"], stats["L"], stats["lin"], stats["Lt0"]) < 1e-12


def test_augmented_truncation_is_the_best_weighted_rank_r_approximation():
    """Eckart-Young in the discrete inner product: the new X S W^T is the best
    rank-r approximation of the rank-2r Galerkin result X_gal L^T, computed here by
    one library SVD of the weighted matrix sqrt(A) psi diag(sqrt(w))."""
    p, quad, grid, st = _warm_augmented(rank=3, nsteps=3)
    r = st.X.shape[1]
    new, stats = O.dlr_step(p, quad, st)
    psi2r = stats["X_gal"] @ stats["L"].T                        # [ncell, nq]
    sa, sw = math.sqrt(grid.area), np.sqrt(quad.w)
    U, s, Vt = np.linalg.svd(sa * psi2r * sw[None, :], full_matrices=False)
    best = (U[:, :r] * s[:r]) @ Vt[:r] / sa / sw[None, :]
    got = new.X @ new.S @ new.W.T
    assert rel(got, best) < 1e-12
    assert np.allclose(stats["sigma_all"], s[:2 * r], rtol=1e-11, atol=1e-14 * s[0])
    assert np.all(s[2 * r:] <= 1e-12 * s[0])                     # the Galerkin result has rank 2r
    assert s[r] > 1e-8 * s[0]                                    # and the truncation is not empty
    err = math.sqrt(grid.area) * np.linalg.norm((psi2r - got) * sw[None, :])
    assert abs(err - np.linalg.norm(s[r:])) < 1e-10 * s[0]
    assert np.max(np.abs(grid.area * new.X.T @ new.X - np.eye(r))) < 1e-13
    assert np.max(np.abs(new.W.T @ (quad.w[:, None] * new.W) - np.eye(r))) < 1e-13


def test_augmented_rank_limit_and_space_exhaustion_raise():
    q = _augmented(_warm_tiny(nx=5, ny=4, npol=2, naz=4, rank=5))   # 2 r = 10 > 8 ordinates
    quad8 = O.quadrature(2, 4)
    st8 = O.dlr_initial_state(q, quad8)
    with pytest.raises(ValueError):
        O.dlr_step(q, quad8, st8)
    rng = np.random.default_rng(0)
    with pytest.raises(ValueError):
        O.cgs2(rng.standard_normal((4, 6)), np.ones(4), O.angular_completion(quad8))
