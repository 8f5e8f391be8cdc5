"""Pins of the bilinear (Q1) upwind DG sweep oracle.

Each pin comes from outside the oracle's own formulas: the exactness of a
Galerkin method on a solution inside its space, the closed-form outflow factor
of the one-dimensional linear DG element (the (1,2) Pade approximant of e^-z),
the paper's own face matrix (central flux plus half the jump penalty) assembled
into one global system and solved directly, the conservation statement of the
weak form with the constant test function (integrals taken by closed-form
quadrature, not by the oracle's matrices), second-order convergence on a smooth
solution, and mirror symmetry.
"""
import math

import numpy as np
import pytest

from oracle import q1_oracle as Q

QUADRANTS = [(0.6, 0.3), (-0.45, 0.7), (0.35, -0.8), (-0.9, -0.25)]


def bilinear(c, x, y):
    return c[0] + c[1] * x + c[2] * y + c[3] * x * y


def manufactured(nx, ny, hx, hy, mu, eta, sigma_t, fun, grad, x0=0.0, y0=0.0):
    """Nodal source s = Omega . grad psi + sigma_t psi and exact inflow data for a given psi."""
    xy = Q.node_coordinates(nx, ny, hx, hy, x0, y0)
    nd = len(mu)
    src = np.empty((nd, nx * ny, 4))
    exact = np.empty((nd, nx * ny, 4))
    inx = np.empty((nd, ny, 2))
    iny = np.empty((nd, nx, 2))
    X, Y = xy[..., 0], xy[..., 1]
    gx, gy = grad(X, Y)
    for d in range(nd):
        exact[d] = fun(X, Y)
        src[d] = mu[d] * gx + eta[d] * gy + sigma_t[:, None] * exact[d]
        xb = x0 if mu[d] > 0 else x0 + nx * hx
        for j in range(ny):
            for iy in range(2):
                inx[d, j, iy] = fun(xb, y0 + (j + iy) * hy)
        yb = y0 if eta[d] > 0 else y0 + ny * hy
        for i in range(nx):
            for ix in range(2):
                iny[d, i, ix] = fun(x0 + (i + ix) * hx, yb)
    return src, inx, iny, exact


@pytest.mark.parametrize("mu,eta", QUADRANTS)
def test_bilinear_solution_is_reproduced(mu, eta):
    """A globally bilinear psi lies in the discrete space and is continuous, so the
    upwind DG solution equals it exactly (per-cell sigma_t keeps the source in Q1)."""
    rng = np.random.default_rng(3)
    nx, ny, hx, hy = 5, 4, 0.3, 0.45
    sig = rng.uniform(0.0, 4.0, nx * ny)
    c = np.array([1.3, -0.7, 0.4, 2.1])
    fun = lambda x, y: bilinear(c, x, y)
    grad = lambda x, y: (c[1] + c[3] * y, c[2] + c[3] * x)
    src, inx, iny, exact = manufactured(nx, ny, hx, hy, [mu], [eta], sig, fun, grad, 0.2, -0.1)
    psi = Q.sweep(nx, ny, hx, hy, np.array([mu]), np.array([eta]), sig, src, inx, iny)
    assert np.max(np.abs(psi - exact)) < 1e-12


def pade_12(z):
    return (1.0 - z / 3.0) / (1.0 + 2.0 * z / 3.0 + z * z / 6.0)


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_one_dimensional_outflow_factor(axis, sign):
    """Pure absorber, unit inflow along one axis and no transport along the other:
    the linear DG element multiplies the outflow value by R(z) = (1 - z/3)/(1 + 2z/3 + z^2/6)
    per cell, z = sigma h / |mu|, and its inflow-side node holds (1 + 2z/3)/(1 + 2z/3 + z^2/6)
    times the incoming value."""
    n, h, sig0, m = 7, 0.4, 1.7, 0.55
    z = sig0 * h / m
    if axis == "x":
        nx, ny, mu, eta = n, 2, sign * m, 0.0
    else:
        nx, ny, mu, eta = 2, n, 0.0, sign * m
    sig = np.full(nx * ny, sig0)
    src = np.zeros((1, nx * ny, 4))
    inx = np.ones((1, ny, 2)) if axis == "x" else np.zeros((1, ny, 2))
    iny = np.ones((1, nx, 2)) if axis == "y" else np.zeros((1, nx, 2))
    psi = Q.sweep(nx, ny, h, h, np.array([mu]), np.array([eta]), sig, src, inx, iny)[0]
    R = pade_12(z)
    R0 = (1.0 + 2.0 * z / 3.0) / (1.0 + 2.0 * z / 3.0 + z * z / 6.0)
    for k in range(n):
        pos = k if sign > 0 else n - 1 - k
        for other in range(2):
            if axis == "x":
                c = other * nx + pos
                a_in, a_out = (0, 1) if sign > 0 else (1, 0)
                nodes = [(a_in, a_out), (a_in + 2, a_out + 2)]
            else:
                c = pos * nx + other
                a_in, a_out = (0, 2) if sign > 0 else (2, 0)
                nodes = [(a_in, a_out), (a_in + 1, a_out + 1)]
            for ai, ao in nodes:
                assert abs(psi[c, ao] - R ** (k + 1)) < 1e-14
                assert abs(psi[c, ai] - R0 * R ** k) < 1e-14


def test_paper_face_matrix_gives_the_same_solution():
    """Assemble (Omega . G + F_d + M_t) psi = M s + inflow terms on the whole mesh with the
    paper's definitions -- G_j = -int dv/dx_j u, and on interior faces the central flux
    -(Omega.n)[[v]]{{u}} plus (1/2)|Omega.n|[[u]][[v]], jumps taken as the value on the side
    n points to minus the value on the side it leaves -- solve it directly, and compare with
    the cell-by-cell upwind sweep.  Boundary faces: outflow on the matrix, inflow data on the
    right-hand side.  Integrals by 2-point Gauss quadrature, independent of the oracle."""
    rng = np.random.default_rng(11)
    nx, ny, hx, hy = 4, 3, 0.5, 0.35
    sig = rng.uniform(0.1, 3.0, nx * ny)
    g = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)])   # Gauss points on [0, 1]
    gw = np.array([0.5, 0.5])

    def basis(a, xi, et):
        bx = xi if a % 2 else 1.0 - xi
        by = et if a // 2 else 1.0 - et
        return bx * by

    def dbasis(a, xi, et):
        bx = xi if a % 2 else 1.0 - xi
        by = et if a // 2 else 1.0 - et
        dx = (1.0 if a % 2 else -1.0) / hx
        dy = (1.0 if a // 2 else -1.0) / hy
        return dx * by, bx * dy

    for mu, eta in QUADRANTS:
        n = 4 * nx * ny
        A = np.zeros((n, n))
        b = np.zeros(n)
        src = rng.standard_normal((nx * ny, 4))
        inx = rng.standard_normal((ny, 2))
        iny = rng.standard_normal((nx, 2))
        for j in range(ny):
            for i in range(nx):
                c = j * nx + i
                for qa in range(2):
                    for qb in range(2):
                        w = gw[qa] * gw[qb] * hx * hy
                        xi, et = g[qa], g[qb]
                        s_q = sum(src[c, bb] * basis(bb, xi, et) for bb in range(4))
                        for a in range(4):
                            va = basis(a, xi, et)
                            dvx, dvy = dbasis(a, xi, et)
                            b[4 * c + a] += w * s_q * va
                            for bb in range(4):
                                ub = basis(bb, xi, et)
                                A[4 * c + a, 4 * c + bb] += w * (-(mu * dvx + eta * dvy) * ub + sig[c] * va * ub)

        def face_points(c, side):
            """Reference coordinates of the face quadrature points in cell c and the face length."""
            if side == "left":
                return [(0.0, t) for t in g], hy
            if side == "right":
                return [(1.0, t) for t in g], hy
            if side == "bottom":
                return [(t, 0.0) for t in g], hx
            return [(t, 1.0) for t in g], hx

        # interior faces: L -> R along +x and +y, normal n from L to R
        faces = []
        for j in range(ny):
            for i in range(nx - 1):
                faces.append((j * nx + i, j * nx + i + 1, "right", "left", mu))
        for j in range(ny - 1):
            for i in range(nx):
                faces.append((j * nx + i, (j + 1) * nx + i, "top", "bottom", eta))
        for cl, cr, sl, sr, on in faces:
            pl, length = face_points(cl, sl)
            pr, _ = face_points(cr, sr)
            for q in range(2):
                w = gw[q] * length
                # [[w]] = w_R - w_L, {{u}} = (u_L + u_R)/2
                vals = {}
                for a in range(4):
                    vals[(cl, a)] = (basis(a, *pl[q]), -1.0)
                    vals[(cr, a)] = (basis(a, *pr[q]), 1.0)
                for (cv, av), (bv, jv) in vals.items():
                    for (cu, au), (bu, ju) in vals.items():
                        term = -on * (jv * bv) * 0.5 * bu + 0.5 * abs(on) * (ju * bu) * (jv * bv)
                        A[4 * cv + av, 4 * cu + au] += w * term
        # boundary faces
        for j in range(ny):
            for side, cell, outward in (("left", j * nx, -1.0), ("right", j * nx + nx - 1, 1.0)):
                on = outward * mu
                pts, length = face_points(cell, side)
                for q in range(2):
                    w = gw[q] * length
                    if on > 0:
                        for a in range(4):
                            for bb in range(4):
                                A[4 * cell + a, 4 * cell + bb] += w * on * basis(a, *pts[q]) * basis(bb, *pts[q])
                    else:
                        gval = inx[j, 0] * (1 - g[q]) + inx[j, 1] * g[q]
                        for a in range(4):
                            b[4 * cell + a] += w * abs(on) * gval * basis(a, *pts[q])
        for i in range(nx):
            for side, cell, outward in (("bottom", i, -1.0), ("top", (ny - 1) * nx + i, 1.0)):
                on = outward * eta
                pts, length = face_points(cell, side)
                for q in range(2):
                    w = gw[q] * length
                    if on > 0:
                        for a in range(4):
                            for bb in range(4):
                                A[4 * cell + a, 4 * cell + bb] += w * on * basis(a, *pts[q]) * basis(bb, *pts[q])
                    else:
                        gval = iny[i, 0] * (1 - g[q]) + iny[i, 1] * g[q]
                        for a in range(4):
                            b[4 * cell + a] += w * abs(on) * gval * basis(a, *pts[q])
        direct = np.linalg.solve(A, b).reshape(nx * ny, 4)
        psi = Q.sweep(nx, ny, hx, hy, np.array([mu]), np.array([eta]), sig, src[None], inx[None], iny[None])[0]
        assert np.max(np.abs(psi - direct)) < 1e-12 * max(1.0, np.max(np.abs(direct)))


def test_conservation_with_constant_test_function():
    """Absorption + boundary outflow = source + boundary inflow, per direction, with cell
    and face integrals of the bilinear fields taken in closed form (node averages)."""
    rng = np.random.default_rng(5)
    nx, ny, hx, hy = 6, 5, 0.25, 0.4
    mu = np.array([q[0] for q in QUADRANTS])
    eta = np.array([q[1] for q in QUADRANTS])
    sig = rng.uniform(0.0, 2.0, nx * ny)
    src = rng.uniform(0.0, 1.0, (4, nx * ny, 4))
    inx = rng.uniform(0.0, 1.0, (4, ny, 2))
    iny = rng.uniform(0.0, 1.0, (4, nx, 2))
    psi = Q.sweep(nx, ny, hx, hy, mu, eta, sig, src, inx, iny)
    area = hx * hy
    for d in range(4):
        absorb = np.sum(sig * area * psi[d].mean(axis=1))
        source = np.sum(area * src[d].mean(axis=1))
        right, left = psi[d][:, [1, 3]].mean(axis=1), psi[d][:, [0, 2]].mean(axis=1)
        top, bottom = psi[d][:, [2, 3]].mean(axis=1), psi[d][:, [0, 1]].mean(axis=1)
        rows_out = (right if mu[d] > 0 else left).reshape(ny, nx)[:, -1 if mu[d] > 0 else 0]
        cols_out = (top if eta[d] > 0 else bottom).reshape(ny, nx)[-1 if eta[d] > 0 else 0, :]
        out = abs(mu[d]) * hy * rows_out.sum() + abs(eta[d]) * hx * cols_out.sum()
        inflow = abs(mu[d]) * hy * inx[d].mean(axis=1).sum() + abs(eta[d]) * hx * iny[d].mean(axis=1).sum()
        assert abs(absorb + out - source - inflow) < 1e-12 * (source + inflow)
        assert abs(Q.boundary_balance(nx, ny, hx, hy, mu[d:d + 1], eta[d:d + 1], sig, src[d:d + 1],
                                      inx[d:d + 1], iny[d:d + 1], psi[d:d + 1])[0]) < 1e-12 * (source + inflow)


def test_second_order_convergence():
    """Smooth solution psi = 2 + sin(pi x) cos(pi y) on the unit square: the nodal error
    falls at least like h^2 under refinement (Q1 elements)."""
    mu, eta, sig0 = np.array([0.7]), np.array([-0.4]), 1.3
    fun = lambda x, y: 2.0 + np.sin(math.pi * x) * np.cos(math.pi * y)
    grad = lambda x, y: (math.pi * np.cos(math.pi * x) * np.cos(math.pi * y),
                         -math.pi * np.sin(math.pi * x) * np.sin(math.pi * y))
    errs = []
    for n in (8, 16, 32):
        h = 1.0 / n
        sig = np.full(n * n, sig0)
        src, inx, iny, exact = manufactured(n, n, h, h, mu, eta, sig, fun, grad)
        psi = Q.sweep(n, n, h, h, mu, eta, sig, src, inx, iny)
        errs.append(np.max(np.abs(psi - exact)))
    assert errs[0] < 0.05
    for a, b in zip(errs, errs[1:]):
        assert a / b > 3.5


def test_mirror_symmetry():
    """Reflecting the problem in x (mu -> -mu, columns reversed, nodes ix swapped)
    reflects the solution."""
    rng = np.random.default_rng(9)
    nx, ny, hx, hy = 5, 4, 0.3, 0.2
    sig = rng.uniform(0.0, 2.0, nx * ny)
    src = rng.standard_normal((1, nx * ny, 4))
    inx = rng.standard_normal((1, ny, 2))
    iny = rng.standard_normal((1, nx, 2))
    psi = Q.sweep(nx, ny, hx, hy, np.array([0.6]), np.array([0.5]), sig, src, inx, iny)

    def mirror_cells(a):
        return a.reshape(a.shape[0], ny, nx, *a.shape[2:])[:, :, ::-1].reshape(a.shape)

    swap = [1, 0, 3, 2]
    src_m = mirror_cells(src)[:, :, swap]
    sig_m = sig.reshape(ny, nx)[:, ::-1].reshape(-1)
    iny_m = iny[:, ::-1, ::-1]
    psi_m = Q.sweep(nx, ny, hx, hy, np.array([-0.6]), np.array([0.5]), sig_m, src_m, inx, iny_m)
    assert np.max(np.abs(mirror_cells(psi_m)[:, :, swap] - psi)) < 1e-13
