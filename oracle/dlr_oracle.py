"""FP64 CPU oracle of the SN-like dynamic low-rank (DLR) method for gray thermal
radiative transfer (Haut, Loffeld, Einkemmer, Guthrey, Brunner, Schill,
arXiv 2601.18705), and of the plain discrete-ordinates (SN) step it reduces to.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module.  The HIP library never
uses it, shares no code with it, and must fail loudly rather than fall back to
it.

It is written to be checked by eye against the paper: plain numpy in float64,
one function per step of Algorithm 1 (the SN-like DLR time step), no fusion and
no reordering beyond what each definition states.  The only compiled piece is
the upwind sweep (``sweep.c``), a forward substitution in plain C loops.
Library primitives used as steps: Gauss-Legendre nodes, small dense solves and
inverses, matrix products, and the SVD of the r x r coupling matrix.

Readings of the paper where it is silent, garbled or inconsistent:
  * B(T) = a c T^4 / (4 pi) (per steradian), so 4 pi B' = 4 a c T^3.
  * Effective source (Newton linearisation of backward Euler for T): the source
    is sigma B(T0) rho c_v / D with D = rho c_v + 4 pi dt sigma B'(T0); the
    printed numerator carries a stray rho c_v T0 term that does not follow
    from the linearisation.  The same stray term is dropped from the
    temperature update T = T0 + dt sigma (phi - 4 pi B(T0)) / D.
  * Spatial discretisation: the degree-0 member of the paper's upwind DG
    family (constants per cell); the L-step uses the same discrete upwind
    operator as the sweep so that full rank reproduces SN exactly.
  * Quadrature: product of n_polar-point Gauss-Legendre in the polar cosine on
    (0, 1) (upper hemisphere; xy symmetry) and n_azim equally spaced
    azimuths (2k-1) pi / n_azim; weights sum to 4 pi.
  * Source iteration starts from the current mean intensity and stops on the
    relative 2-norm change of phi (plus the change of Psi when a side reflects).
  * "Stabilised Gram-Schmidt" = classical Gram-Schmidt with one
    reorthogonalisation (CGS2); rank-deficient columns are replaced by the next
    graded monomial completion vector.
  * DEIM ties: among nodes with |R| >= (1 - tau) max |R| the smallest index wins.
  * After the L-step QR, an SVD of S = U Sigma V^T rotates X <- X U, W <- W V,
    S <- Sigma (rank stays r); V columns are signed so that their
    largest-magnitude entry is positive.
  * Initial factors: psi(0) = B(T_init) isotropic, completed by monomials.
  * Reflecting walls: the inflow is the outflow of the mirrored direction,
    lagged inside the source iteration (collocation directions interpolate it
    through W) and inside a fixed-point iteration of the L-step.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import build_oracle

FOUR_PI = 4.0 * math.pi
BC_VACUUM, BC_INFLOW, BC_REFLECT = 0, 1, 2
SIDE_LEFT, SIDE_RIGHT, SIDE_BOTTOM, SIDE_TOP = 0, 1, 2, 3

_lib = None


def _sweep_lib():
    global _lib
    if _lib is None:
        path = build_oracle.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
        lib.oracle_sweep.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# =========================================================================== grid and quadrature

@dataclass
class Grid:
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float

    @property
    def hx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def hy(self):
        return (self.y1 - self.y0) / self.ny

    @property
    def area(self):
        return self.hx * self.hy

    @property
    def ncell(self):
        return self.nx * self.ny

    def side_mask(self, side):
        """Indicator of the cells adjacent to one side of the domain."""
        m = np.zeros((self.ny, self.nx))
        if side == SIDE_LEFT:
            m[:, 0] = 1.0
        elif side == SIDE_RIGHT:
            m[:, -1] = 1.0
        elif side == SIDE_BOTTOM:
            m[0, :] = 1.0
        else:
            m[-1, :] = 1.0
        return m.ravel()


def grid_of(p):
    return Grid(p["nx"], p["ny"], p["x0"], p["x1"], p["y0"], p["y1"])


@dataclass
class Quadrature:
    mu: np.ndarray      # x direction cosine
    eta: np.ndarray     # y direction cosine
    xi: np.ndarray      # polar cosine (z), in (0, 1)
    w: np.ndarray       # weights, sum 4 pi
    refl_x: np.ndarray  # index of (-mu, eta)
    refl_y: np.ndarray  # index of (mu, -eta)

    @property
    def n(self):
        return self.mu.size


def quadrature(n_polar, n_azim):
    """Product Gauss-Legendre (polar cosine on (0,1)) x equally spaced azimuths.

    Index q = p * n_azim + k.  The ordinate set is closed under mu -> -mu and
    eta -> -eta when n_azim is even; n_azim % 4 == 0 keeps mu and eta non-zero.
    """
    if n_azim % 4 != 0:
        raise ValueError("n_azim must be a multiple of 4")
    x, wgl = np.polynomial.legendre.leggauss(n_polar)
    xi = 0.5 * (1.0 + x)
    om = 0.5 * wgl
    phi = (2.0 * np.arange(1, n_azim + 1) - 1.0) * math.pi / n_azim
    XI, PHI = np.meshgrid(xi, phi, indexing="ij")
    OM = np.repeat(om[:, None], n_azim, axis=1)
    s = np.sqrt(1.0 - XI ** 2)
    mu = (s * np.cos(PHI)).ravel()
    eta = (s * np.sin(PHI)).ravel()
    w = (FOUR_PI * OM / n_azim).ravel()
    xi_f = XI.ravel()

    def mirror(mx, my):
        idx = np.empty(mu.size, dtype=np.int64)
        for q in range(mu.size):
            d = (mu - mx * mu[q]) ** 2 + (eta - my * eta[q]) ** 2 + (xi_f - xi_f[q]) ** 2
            idx[q] = int(np.argmin(d))
        return idx

    return Quadrature(mu, eta, xi_f, w, mirror(-1.0, 1.0), mirror(1.0, -1.0))


# =========================================================================== physics (Sec. 2)

def planck(T, a, c):
    """B(T) = a c T^4 / (4 pi): equilibrium intensity per steradian."""
    return a * c * T ** 4 / FOUR_PI


def planck_dT(T, a, c):
    return a * c * T ** 3 / math.pi


@dataclass
class Linearised:
    D: np.ndarray        # rho c_v + 4 pi dt sigma dB/dT
    sigma_s: np.ndarray  # pseudo-scattering opacity
    q: np.ndarray        # effective isotropic source per steradian (incl. external)
    sigma_t: np.ndarray  # sigma + 1/(c dt)
    emis0: np.ndarray    # 4 pi B(T0)


def linearise(p, T0):
    """Newton linearisation of the backward-Euler temperature equation
    (eq. "effective scattering" and "effective source", read as described in
    the module docstring)."""
    sig, rcv, dt, a, c = p["sigma_a"], p["rho_cv"], p["dt"], p["a"], p["c"]
    B0 = planck(T0, a, c)
    dB0 = planck_dT(T0, a, c)
    D = rcv + FOUR_PI * dt * sig * dB0
    sigma_s = (FOUR_PI * dt * sig * dB0 / D) * sig
    q = sig * B0 * rcv / D + p["q_ext"] / FOUR_PI
    sigma_t = sig + 1.0 / (c * dt)
    return Linearised(D, sigma_s, q, sigma_t, FOUR_PI * B0)


def temperature_update(p, T0, lin, phi):
    """eq. "temperature update": T = T0 + dt sigma (phi - 4 pi B(T0)) / D."""
    return T0 + p["dt"] * p["sigma_a"] * (phi - lin.emis0) / lin.D


def total_energy(p, grid, T, phi):
    """Sum over cells of area * (rho c_v T + phi / c)."""
    return float(grid.area * np.sum(p["rho_cv"] * T + phi / p["c"]))


def source_power(p, grid):
    """Sum over cells of area * q_ext (q_ext is the angle-integrated external source)."""
    return float(grid.area * np.sum(p["q_ext"]))


def boundary_flows(p, grid, quad, side_psi):
    """Radiation power entering and leaving through the sides of the domain.

    side_psi(side) -> [nq, m]: the intensity of every ordinate on the m cells
    along that side (row order on the left and right, column order on the
    bottom and top).  Summing the degree-0 upwind equations over cells and
    ordinates (weights w_q, cell area) telescopes each row and column of the
    transport term to its two end faces, so a face contributes
    w_q |Omega_q . n| psi_face times its length (h_y on the left and right
    sides, h_x on the bottom and top).  Leaving: the wall cell's own value
    (the upwind trace) for ordinates with Omega . n > 0.  Entering: the inflow
    value -- B(T_b) on an INFLOW side, 0 on a VACUUM side, the mirrored
    ordinate's wall value on a REFLECT side.  With these,
      E_tot(new) - E_tot(old) = dt (source_power + inflow - outflow)
    holds exactly for plain SN and full-rank DLR (time-discrete balance of the
    temperature update and the transport equation of Sec. 2).

    Returns (inflow, outflow)."""
    face = {SIDE_LEFT: grid.hy, SIDE_RIGHT: grid.hy, SIDE_BOTTOM: grid.hx, SIDE_TOP: grid.hx}
    inflow = 0.0
    outflow = 0.0
    for side in range(4):
        vals = side_psi(side)
        if side in (SIDE_LEFT, SIDE_RIGHT):
            cosn = quad.mu if side == SIDE_RIGHT else -quad.mu     # Omega . n, outward normal
            mirror = quad.refl_x
        else:
            cosn = quad.eta if side == SIDE_TOP else -quad.eta
            mirror = quad.refl_y
        for qi in range(quad.n):
            if cosn[qi] > 0.0:
                outflow += quad.w[qi] * cosn[qi] * face[side] * float(np.sum(vals[qi]))
            else:
                kind = p["bc"][side]
                if kind == BC_INFLOW:
                    psib = planck(p["T_b"][side], p["a"], p["c"])
                    inflow += quad.w[qi] * (-cosn[qi]) * face[side] * psib * vals.shape[1]
                elif kind == BC_REFLECT:
                    inflow += quad.w[qi] * (-cosn[qi]) * face[side] * float(np.sum(vals[mirror[qi]]))
    return inflow, outflow


def side_cells(grid, side):
    """Cell indices (e = j nx + i) along one side, in row or column order."""
    e = np.arange(grid.ncell).reshape(grid.ny, grid.nx)
    if side == SIDE_LEFT:
        return e[:, 0]
    if side == SIDE_RIGHT:
        return e[:, -1]
    if side == SIDE_BOTTOM:
        return e[0, :]
    return e[-1, :]


# =========================================================================== sweep + inflow

def sweep(grid, mu, eta, sigma_t, rhs, inx, iny):
    """Invert the degree-0 upwind operator + sigma_t for each direction.

    rhs [nd, ncell], inx [nd, ny], iny [nd, nx] -> psi [nd, ncell]."""
    nd = mu.size
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    inx = np.ascontiguousarray(inx, dtype=np.float64)
    iny = np.ascontiguousarray(iny, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    st = np.ascontiguousarray(sigma_t, dtype=np.float64)
    psi = np.empty((nd, grid.ncell))
    _sweep_lib().oracle_sweep(grid.nx, grid.ny, grid.hx, grid.hy, nd, _ptr(mu), _ptr(eta), _ptr(st),
                              _ptr(rhs), _ptr(inx), _ptr(iny), _ptr(psi))
    return psi


def x_inflow_side(mu):
    return SIDE_LEFT if mu > 0 else SIDE_RIGHT


def y_inflow_side(eta):
    return SIDE_BOTTOM if eta > 0 else SIDE_TOP


def wall_values(grid, field2d, side):
    """Values of a [ncell] field on the cells along one side (row/column order)."""
    f = field2d.reshape(grid.ny, grid.nx)
    if side == SIDE_LEFT:
        return f[:, 0]
    if side == SIDE_RIGHT:
        return f[:, -1]
    if side == SIDE_BOTTOM:
        return f[0, :]
    return f[-1, :]


def inflow_arrays(p, grid, mu, eta, reflected):
    """Inflow face values for directions (mu, eta).

    reflected(d, side) -> wall-cell values of the mirrored direction, called
    only for reflecting sides."""
    nd = mu.size
    inx = np.zeros((nd, grid.ny))
    iny = np.zeros((nd, grid.nx))
    for d in range(nd):
        sx = x_inflow_side(mu[d])
        sy = y_inflow_side(eta[d])
        for side, arr in ((sx, inx), (sy, iny)):
            kind = p["bc"][side]
            if kind == BC_INFLOW:
                arr[d, :] = planck(p["T_b"][side], p["a"], p["c"])
            elif kind == BC_REFLECT:
                arr[d, :] = reflected(d, side)
    return inx, iny


def any_reflecting(p):
    return any(b == BC_REFLECT for b in p["bc"])


# =========================================================================== plain SN step

@dataclass
class SNState:
    T: np.ndarray
    psi: np.ndarray     # [nq, ncell]
    phi: np.ndarray


def sn_initial_state(p, quad):
    B0 = planck(p["T_init"], p["a"], p["c"])
    psi = np.repeat(B0[None, :], quad.n, axis=0)
    return SNState(p["T_init"].copy(), psi, FOUR_PI * B0)


def sn_step(p, quad, st, tol=None, max_iter=None):
    """One backward-Euler step of plain SN with source iteration over all
    ordinates (the method the SN-like DLR step reproduces at full rank)."""
    grid = grid_of(p)
    tol = p["si_tol"] if tol is None else tol
    max_iter = p["si_max_iter"] if max_iter is None else max_iter
    lin = linearise(p, st.T)
    cdt = p["c"] * p["dt"]
    fixed = lin.q[None, :] + st.psi / cdt
    phi = quad.w @ st.psi
    psi_prev = st.psi
    refl = any_reflecting(p)
    it = 0
    while True:
        it += 1
        rhs = lin.sigma_s[None, :] * phi[None, :] / FOUR_PI + fixed

        def reflected(d, side, _prev=psi_prev):
            m = quad.refl_x[d] if side in (SIDE_LEFT, SIDE_RIGHT) else quad.refl_y[d]
            return wall_values(grid, _prev[m], side)

        inx, iny = inflow_arrays(p, grid, quad.mu, quad.eta, reflected)
        psi = sweep(grid, quad.mu, quad.eta, lin.sigma_t, rhs, inx, iny)
        phi_new = quad.w @ psi
        dphi = np.linalg.norm(phi_new - phi)
        ok = dphi <= tol * np.linalg.norm(phi_new)
        if refl:
            ok = ok and np.linalg.norm(psi - psi_prev) <= tol * np.linalg.norm(psi)
        if p.get("dsa") and not ok:
            phi_next = dsa_correct(grid, lin, dsa_kappas(quad.w, quad.mu, quad.eta), phi_new, phi)
        else:
            phi_next = phi_new
        phi, psi_prev = phi_next, psi
        if ok:
            break
        if it >= max_iter:
            raise RuntimeError("plain SN source iteration did not converge")
    T = temperature_update(p, st.T, lin, phi)
    inflow, outflow = boundary_flows(p, grid, quad, lambda side: psi[:, side_cells(grid, side)])
    return SNState(T, psi, phi), {"si_iters": it, "inflow": inflow, "outflow": outflow,
                                  "energy": total_energy(p, grid, T, phi)}


# =========================================================================== diffusion synthetic acceleration

def dsa_face_operators(grid):
    """Central face operators F_x, F_y of the degree-0 elements: the part of the paper's face
    matrix F_d that is linear in Omega (Sec. 4.4, F_d = Omega . F + F_d^[[]], and its DSA appendix),
    v^T F_j u = - sum_faces h_f n_j [[v]] {{u}}, with [[v]] = v_minus - v_plus across a face of
    normal n from the minus to the plus cell, {{u}} the face average, and exterior values 0
    (reading: the boundary treatment is not printed; the error equation of source iteration has
    homogeneous boundary data).  Degree-0 elements have no volume gradient term (G_j = 0).
    Returns scipy sparse [ncell, ncell] matrices, cells e = j*nx + i."""
    import scipy.sparse as sp
    nx, ny = grid.nx, grid.ny
    ops = []
    for axis in (0, 1):
        rows, cols, vals = [], [], []
        h = grid.hy if axis == 0 else grid.hx      # face length
        nfaces = (nx + 1, ny) if axis == 0 else (nx, ny + 1)
        for b in range(nfaces[1]):
            for a in range(nfaces[0]):
                # face between the minus cell (index a-1 along the axis) and the plus cell (index a)
                if axis == 0:
                    minus = b * nx + (a - 1) if a > 0 else None
                    plus = b * nx + a if a < nx else None
                else:
                    minus = (b - 1) * nx + a if b > 0 else None      # here b runs over faces along y
                    plus = b * nx + a if b < ny else None
                cells = [(minus, 1.0), (plus, -1.0)]              # [[v]] weights
                for tv, jv in cells:
                    if tv is None:
                        continue
                    for tu in (minus, plus):
                        if tu is None:
                            continue
                        rows.append(tv)
                        cols.append(tu)
                        vals.append(-h * jv * 0.5)
        ops.append(sp.csr_matrix((vals, (rows, cols)), shape=(grid.ncell, grid.ncell)))
    return ops[0], ops[1]


def dsa_penalty(grid, kappa_x, kappa_y):
    """F_0 of eq. "penalty term": v^T F_0 u = (1/4pi) sum_faces (1/2) kappa_f h_f [[u]][[v]], with
    kappa_f = sum_d c_d |Omega_d . n_f| (c = beta^T What^{-1}, the collocation weights), exterior
    values 0."""
    import scipy.sparse as sp
    nx, ny = grid.nx, grid.ny
    rows, cols, vals = [], [], []

    def face(minus, plus, coef):
        ends = [(minus, 1.0), (plus, -1.0)]
        for tv, jv in ends:
            if tv is None:
                continue
            for tu, ju in ends:
                if tu is None:
                    continue
                rows.append(tv)
                cols.append(tu)
                vals.append(coef * jv * ju)

    cx = kappa_x * grid.hy / (2.0 * FOUR_PI)
    cy = kappa_y * grid.hx / (2.0 * FOUR_PI)
    for j in range(ny):
        for a in range(nx + 1):
            face(j * nx + a - 1 if a > 0 else None, j * nx + a if a < nx else None, cx)
    for b in range(ny + 1):
        for i in range(nx):
            face((b - 1) * nx + i if b > 0 else None, b * nx + i if b < ny else None, cy)
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.ncell, grid.ncell))


def dsa_matrix(grid, sigma_t, sigma_s, kappa_x, kappa_y):
    """The DSA matrix of the appendix derivation for degree-0 elements:
    (1/3) sum_j F_j^T M_t^{-1} F_j + F_0 + M_a, with M_t = area sigma_t, M_a = area (sigma_t - sigma_s)
    (sigma_t includes 1/(c dt) and sigma_s is the pseudo-scattering of the linearisation)."""
    import scipy.sparse as sp
    A = grid.area
    Fx, Fy = dsa_face_operators(grid)
    Mt_inv = sp.diags(1.0 / (A * sigma_t))
    D = (Fx.T @ Mt_inv @ Fx + Fy.T @ Mt_inv @ Fy) / 3.0
    D = D + dsa_penalty(grid, kappa_x, kappa_y) + sp.diags(A * (sigma_t - sigma_s))
    return sp.csr_matrix(D)


def dsa_kappas(cw, mu, eta):
    """kappa_x = sum_d c_d |mu_d|, kappa_y = sum_d c_d |eta_d| (face normals along x and y)."""
    return float(np.dot(cw, np.abs(mu))), float(np.dot(cw, np.abs(eta)))


def dsa_correct(grid, lin, kappa, phi_half, phi_old):
    """One DSA step of source iteration: the transport sweep took phi_old to phi_half; the
    diffusion approximation of the remaining error, D delta = M_s (phi_half - phi_old), is added:
    returns phi_half + delta (exact sparse solve)."""
    import scipy.sparse.linalg as spla
    D = dsa_matrix(grid, lin.sigma_t, lin.sigma_s, *kappa)
    rhs = grid.area * lin.sigma_s * (phi_half - phi_old)
    return phi_half + spla.spsolve(D.tocsc(), rhs)


# =========================================================================== DLR helpers

def spatial_completion(grid):
    """Graded monomials 1, x, y, x^2, xy, y^2, ... at cell centres mapped to [-1,1]^2 (lazy)."""
    xc = -1.0 + (np.arange(grid.nx) + 0.5) * 2.0 / grid.nx
    yc = -1.0 + (np.arange(grid.ny) + 0.5) * 2.0 / grid.ny
    Xc, Yc = np.meshgrid(xc, yc)
    Xc, Yc = Xc.ravel(), Yc.ravel()
    deg = 0
    while True:
        for ax in range(deg, -1, -1):
            yield Xc ** ax * Yc ** (deg - ax)
        deg += 1


def angular_completion(quad):
    """Graded monomials 1, mu, eta, mu^2, mu eta, eta^2, ... on the ordinates (lazy)."""
    deg = 0
    while True:
        for ax in range(deg, -1, -1):
            yield quad.mu ** ax * quad.eta ** (deg - ax)
        deg += 1


def cgs2(V, weight, completion, defect_tol=1e-12, skip_tol=1e-10):
    """Weighted classical Gram-Schmidt with one reorthogonalisation.

    V [n, r] -> Q [n, r], R [r, r] with V = Q R, Q^T diag(weight) Q = I, R upper
    triangular with R_kk >= 0.  A column whose residual norm is at most
    defect_tol times its own norm is replaced by the next completion vector
    (orthogonalised twice, skipped when dependent) and gets R_kk = 0; r > n raises
    ValueError, since the completion could never fill the missing columns.
    (The accepted columns are kept as contiguous rows of Qt = Q^T.)
    """
    n, r = V.shape
    Qt = np.zeros((r, n))
    R = np.zeros((r, r))
    comp = iter(completion)

    def ip(u, v):
        return float(np.dot(weight * u, v))

    def project_out(v, k):
        h = Qt[:k] @ (weight * v)
        return v - Qt[:k].T @ h, h

    for k in range(r):
        v = V[:, k].astype(np.float64)
        own = math.sqrt(max(ip(v, v), 0.0))
        v1, h1 = project_out(v, k)
        v2, h2 = project_out(v1, k)
        R[:k, k] = h1 + h2
        nrm = math.sqrt(max(ip(v2, v2), 0.0))
        if own > 0.0 and nrm > defect_tol * own:
            Qt[k] = v2 / nrm
            R[k, k] = nrm
            continue
        if k >= n:
            raise ValueError(f"cgs2: {r} columns do not fit a space of dimension {n}")
        while True:
            u = next(comp)
            un = math.sqrt(ip(u, u))
            u1, _ = project_out(u, k)
            u2, _ = project_out(u1, k)
            n2 = math.sqrt(max(ip(u2, u2), 0.0))
            if n2 > skip_tol * un:
                Qt[k] = u2 / n2
                R[k, k] = 0.0
                break
    return Qt.T, R


def deim(W, tie_tol, edges=False):
    """Greedy DEIM interpolation points on the angular basis (Sec. 4.2).

    Point j maximises |R_j| where R_j is W_j minus its interpolant by
    W_1..W_{j-1} at the points already chosen.  Near ties (within tie_tol of
    the maximum) go to the smallest ordinate index.  Returns the point indices
    and, per pick, the relative margin to the best non-tied competitor.  With
    edges=True it also returns, per pick, how far the decision is from
    changing: the smallest distance of any |R_q| / max |R| from the tie
    threshold 1 - tie_tol (a perturbation of R smaller than that, relative to
    max |R|, cannot change the pick).
    """
    n, r = W.shape
    sel = []
    margins = []
    edge = []
    for j in range(r):
        if j == 0:
            R = W[:, 0].copy()
        else:
            coef = np.linalg.solve(W[sel, :j], W[sel, j])
            R = W[:, j] - W[:, :j] @ coef
        a = np.abs(R)
        m = a.max()
        tied = a >= (1.0 - tie_tol) * m
        pj = int(np.nonzero(tied)[0].min())
        rest = a[~tied]
        margins.append(float((m - rest.max()) / m) if rest.size else 1.0)
        others = np.delete(a, int(np.argmax(a)))
        edge.append(float(np.min(np.abs(others / m - (1.0 - tie_tol)))) if others.size else 1.0)
        sel.append(pj)
    if edges:
        return np.array(sel, dtype=np.int64), np.array(margins), np.array(edge)
    return np.array(sel, dtype=np.int64), np.array(margins)


@dataclass
class DLRState:
    X: np.ndarray   # [ncell, r], <X_i, X_j> = delta_ij (cell-area weighted)
    S: np.ndarray   # [r, r]
    W: np.ndarray   # [nq, r], sum_q w_q W_qi W_qj = delta_ij
    T: np.ndarray   # [ncell]


def dlr_initial_state(p, quad):
    """psi(0) = B(T_init), isotropic: rank one, completed by monomials."""
    grid = grid_of(p)
    r = p["rank"]
    B0 = planck(p["T_init"], p["a"], p["c"])
    Vx = np.zeros((grid.ncell, r))
    Vx[:, 0] = B0
    X, Rx = cgs2(Vx, np.full(grid.ncell, grid.area), spatial_completion(grid))
    Vw = np.zeros((quad.n, r))
    Vw[:, 0] = 1.0
    W, Rw = cgs2(Vw, quad.w, angular_completion(quad))
    S = np.zeros((r, r))
    S[0, 0] = Rx[0, 0] * Rw[0, 0]
    return DLRState(X, S, W, p["T_init"].copy())


def mean_intensity(quad, st):
    """phi = int psi dOmega = X S (W^T w)."""
    return st.X @ (st.S @ (st.W.T @ quad.w))


def shift_from(grid, U, di, dj):
    """(shift U)_e = U at cell (i - di, j - dj), zero outside the domain. U [ncell, k]."""
    k = U.shape[1]
    V = U.reshape(grid.ny, grid.nx, k)
    out = np.zeros_like(V)
    ys = slice(max(dj, 0), grid.ny + min(dj, 0))
    yd = slice(max(-dj, 0), grid.ny + min(-dj, 0))
    xs = slice(max(di, 0), grid.nx + min(di, 0))
    xd = slice(max(-di, 0), grid.nx + min(-di, 0))
    out[ys, xs] = V[yd, xd]
    return out.reshape(grid.ncell, k)


def upwind_difference_ops(grid, X):
    """D_x^{+-} X and D_y^{+-} X: one-sided differences toward the upwind
    neighbour (zero outside), scaled by 1/h."""
    return {
        "x+": (X - shift_from(grid, X, 1, 0)) / grid.hx,
        "x-": (X - shift_from(grid, X, -1, 0)) / grid.hx,
        "y+": (X - shift_from(grid, X, 0, 1)) / grid.hy,
        "y-": (X - shift_from(grid, X, 0, -1)) / grid.hy,
    }


# =========================================================================== the DLR step (Algorithm 1)

def dlr_step(p, quad, st, forced_sel=None, tol=None, max_iter=None, lstep_tol=1e-14):
    """One SN-like DLR time step, Algorithm 1 steps 1-9, plus the SVD rotation.

    With p["augment"] set, the augmented variant: step 5 orthonormalises the swept
    columns together with the old basis X0 (rank 2r, so the old solution lies in the
    Galerkin space), steps 6-8 run on that basis, and the SVD of step 8 truncates the
    rank-2r result back to its r largest singular values -- the rank-2r -> r truncation
    of the paper's PN-like scheme (Sec. 3, the updated solution of rank 2r and its
    truncated SVD) applied to the SN-like step.

    Returns the new state and a stats dict (SI iterations, DEIM picks/margins,
    singular values, DEIM weights)."""
    grid = grid_of(p)
    tol = p["si_tol"] if tol is None else tol
    max_iter = p["si_max_iter"] if max_iter is None else max_iter
    A = grid.area
    cdt = p["c"] * p["dt"]
    X0, S0, W0, T0 = st.X, st.S, st.W, st.T
    r = X0.shape[1]

    def ip(U, V):
        """<U_i, V_j>_X for the columns of U [ncell, a] and V [ncell, b]."""
        return A * (U.T @ V)

    # 1. effective scattering and source
    lin = linearise(p, T0)

    # 2. DEIM angle selection on W0
    if forced_sel is None:
        sel, margins, edges = deim(W0, p["deim_tie_tol"], edges=True)
    else:
        sel, margins, edges = np.asarray(forced_sel, dtype=np.int64), np.zeros(r), np.zeros(r)
    What = W0[sel, :]                    # What[i, j] = W_j(Omega^(i))
    beta = W0.T @ quad.w                 # beta_j = int W_j
    cw = np.linalg.solve(What.T, beta)   # phi = beta^T What^{-1} Psi = cw . Psi
    mu_s, eta_s = quad.mu[sel], quad.eta[sel]

    # 3. initial condition at the new angles: psi_j^(0) = sum_k L0_k(Omega^(j)) X0_k
    L0 = W0 @ S0.T                       # L0[q, k] = L0_k(Omega_q)
    Psi0 = (X0 @ L0[sel, :].T).T         # [r, ncell]

    # 4. source iteration with sweeps on the collocation system
    fixed = lin.q[None, :] + Psi0 / cdt
    phi = X0 @ (S0 @ beta)
    Psi_prev = Psi0
    refl = any_reflecting(p)
    What_inv = np.linalg.inv(What)
    it = 0
    while True:
        it += 1
        rhs = lin.sigma_s[None, :] * phi[None, :] / FOUR_PI + fixed

        def reflected(d, side, _prev=Psi_prev):
            m = quad.refl_x[sel[d]] if side in (SIDE_LEFT, SIDE_RIGHT) else quad.refl_y[sel[d]]
            K = What_inv @ _prev          # K [r, ncell]
            return wall_values(grid, W0[m, :] @ K, side)

        inx, iny = inflow_arrays(p, grid, mu_s, eta_s, reflected)
        Psi = sweep(grid, mu_s, eta_s, lin.sigma_t, rhs, inx, iny)
        phi_new = cw @ Psi
        ok = np.linalg.norm(phi_new - phi) <= tol * np.linalg.norm(phi_new)
        if refl:
            ok = ok and np.linalg.norm(Psi - Psi_prev) <= tol * np.linalg.norm(Psi)
        if p.get("dsa") and not ok:
            # diffusion synthetic acceleration of the collocation source iteration (Sec. 4, DSA)
            phi_next = dsa_correct(grid, lin, dsa_kappas(cw, mu_s, eta_s), phi_new, phi)
        else:
            phi_next = phi_new
        phi, Psi_prev = phi_next, Psi
        if ok:
            break
        if it >= max_iter:
            raise RuntimeError("DLR source iteration did not converge")

    # 5. orthonormalise the swept columns: Psi = X R
    X, _ = cgs2(Psi.T, np.full(grid.ncell, A), spatial_completion(grid))
    X_pre = X
    augment = bool(p.get("augment"))
    if augment:
        # the swept basis and the old one, orthonormalised together: 2r columns
        if 2 * r > min(quad.n, grid.ncell):
            raise ValueError("augmented step needs 2 r <= min(ordinates, cells)")
        X, _ = cgs2(np.hstack([X, X0]), np.full(grid.ncell, A), spatial_completion(grid))

    X_gal = X

    # 6. project the old solution onto the new spatial basis: Lt0_j = sum_i L0_i <X0_i, X_j>
    P = ip(X0, X)
    Lt0 = L0 @ P

    # 7. L-step (row constraints), Schur complement on the scattering coupling
    L = l_step(p, grid, quad, X, lin, Lt0, cdt, lstep_tol)

    # 8. orthonormalise L = W S^T in the quadrature inner product, then rotate by the SVD of S
    W, R = cgs2(L, quad.w, angular_completion(quad))
    X, S, W = svd_rotate(X, R.T, W)
    sig_all = np.diag(S).copy()
    if augment:
        # truncated SVD: the r largest singular values and their vectors
        X, S, W = X[:, :r], S[:r, :r], W[:, :r]
    sig = np.diag(S).copy()

    # 9. temperature update with the new mean intensity
    new = DLRState(X, S, W, T0)
    phi_new = mean_intensity(quad, new)
    new.T = temperature_update(p, T0, lin, phi_new)
    G = S @ W.T                          # psi on any set of cells = X[cells] G
    inflow, outflow = boundary_flows(p, grid, quad, lambda side: (X[side_cells(grid, side)] @ G).T)
    stats = {"si_iters": it, "sel": sel, "margins": margins, "deim_edge": edges, "sigma": sig,
             "sigma_all": sig_all, "cw": cw,
             "inflow": inflow, "outflow": outflow, "energy": total_energy(p, grid, new.T, phi_new),
             "phi": phi_new, "sum_abs_cw_over_4pi": float(np.abs(cw).sum() / FOUR_PI),
             "Psi": Psi, "Psi0": Psi0, "X_pre": X_pre, "X_gal": X_gal, "L": L, "lin": lin, "Lt0": Lt0}
    return new, stats


def svd_rotate(X, S, W):
    """S = U Sigma V^T (singular values descending); return X U, Sigma, W V.

    psi = X S W^T is unchanged.  Each V column is signed so that its
    largest-magnitude entry is positive (U follows)."""
    U, sig, Vt = np.linalg.svd(S)
    V = Vt.T.copy()
    U = U.copy()
    for k in range(S.shape[0]):
        m = int(np.argmax(np.abs(V[:, k])))
        if V[m, k] < 0.0:
            V[:, k] = -V[:, k]
            U[:, k] = -U[:, k]
    return X @ U, np.diag(sig), W @ V


def l_step(p, grid, quad, X, lin, Lt0, cdt, tol):
    """Solve (A(Omega) + M_t) L = M_s (int L dOmega) / (4 pi) + Q for every ordinate.

    A(Omega) = <X, T_Omega X> with the sweep's own upwind operator T_Omega =
    |mu| D_x^{sgn mu} + |eta| D_y^{sgn eta}; inflow faces contribute to Q.  The
    isotropic coupling is removed with the Schur complement used for the
    PN-like L step: Cbar = sum_q w_q B_q^{-1}, zeta = sum_q w_q B_q^{-1} Q_q,
    (I - Cbar M_s / (4 pi)) Lbar = zeta, then L_q = B_q^{-1}(M_s Lbar/(4 pi) + Q_q).
    Reflecting walls add the mirrored ordinate's L on the right-hand side,
    iterated to a fixed point.
    """
    A = grid.area
    r = X.shape[1]
    nq = quad.n

    def ip(U, V):
        return A * (U.T @ V)

    D = upwind_difference_ops(grid, X)
    Ax = {1: ip(X, D["x+"]), -1: ip(X, D["x-"])}
    Ay = {1: ip(X, D["y+"]), -1: ip(X, D["y-"])}
    Mt = ip(X, lin.sigma_t[:, None] * X)
    Ms = ip(X, lin.sigma_s[:, None] * X)
    qX = ip(X, lin.q[:, None])[:, 0]
    hside = {SIDE_LEFT: grid.hx, SIDE_RIGHT: grid.hx, SIDE_BOTTOM: grid.hy, SIDE_TOP: grid.hy}
    bvec = {s: ip(X, grid.side_mask(s)[:, None])[:, 0] / hside[s] for s in range(4)}
    Eside = {s: ip(X, grid.side_mask(s)[:, None] * X) / hside[s] for s in range(4)}

    B = np.empty((nq, r, r))
    Q = np.empty((nq, r))
    for q in range(nq):
        mu, eta = quad.mu[q], quad.eta[q]
        sx, sy = (1 if mu > 0 else -1), (1 if eta > 0 else -1)
        B[q] = abs(mu) * Ax[sx] + abs(eta) * Ay[sy] + Mt
        Q[q] = qX + Lt0[q] / cdt
        for side, cosn in ((x_inflow_side(mu), abs(mu)), (y_inflow_side(eta), abs(eta))):
            if p["bc"][side] == BC_INFLOW:
                Q[q] += cosn * planck(p["T_b"][side], p["a"], p["c"]) * bvec[side]

    Binv = np.linalg.inv(B)
    Cbar = np.einsum("q,qij->ij", quad.w, Binv)
    schur = np.eye(r) - Cbar @ Ms / FOUR_PI

    def solve_with(Qq):
        zeta = np.einsum("q,qij,qj->i", quad.w, Binv, Qq)
        Lbar = np.linalg.solve(schur, zeta)
        rhs = (Ms @ Lbar / FOUR_PI)[None, :] + Qq
        return np.linalg.solve(B, rhs[:, :, None])[:, :, 0]

    if not any_reflecting(p):
        return solve_with(Q)

    L = Lt0.copy()
    for _ in range(100000):
        Qr = Q.copy()
        for q in range(nq):
            mu, eta = quad.mu[q], quad.eta[q]
            for side, cosn, m in ((x_inflow_side(mu), abs(mu), quad.refl_x[q]),
                                  (y_inflow_side(eta), abs(eta), quad.refl_y[q])):
                if p["bc"][side] == BC_REFLECT:
                    Qr[q] += cosn * (Eside[side] @ L[m])
        Ln = solve_with(Qr)
        done = np.linalg.norm(Ln - L) <= tol * np.linalg.norm(Ln)
        L = Ln
        if done:
            return L
    raise RuntimeError("reflecting L-step did not converge")


# =========================================================================== drivers

def run_dlr(p, nsteps=None, forced=None, record=True):
    """Run the DLR method; returns the final state and per-step records
    (E_r = phi / c, T, stats)."""
    quad = quadrature(p["n_polar"], p["n_azim"])
    st = dlr_initial_state(p, quad)
    nsteps = p["nsteps"] if nsteps is None else nsteps
    hist = []
    for n in range(nsteps):
        fs = None if forced is None else forced[n]
        st, stats = dlr_step(p, quad, st, forced_sel=fs)
        if record:
            hist.append({"E_r": stats["phi"] / p["c"], "T": st.T.copy(), **stats})
    return st, hist


def run_sn(p, nsteps=None):
    quad = quadrature(p["n_polar"], p["n_azim"])
    st = sn_initial_state(p, quad)
    nsteps = p["nsteps"] if nsteps is None else nsteps
    hist = []
    for n in range(nsteps):
        st, stats = sn_step(p, quad, st)
        hist.append({"E_r": st.phi / p["c"], "T": st.T.copy(), **stats})
    return st, hist
