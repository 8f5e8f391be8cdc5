"""FP64 CPU oracle of the bilinear (Q1) upwind discontinuous-Galerkin transport
sweep -- the spatial discretisation the paper states for the collocation solve
(Sec. "Spatial discretization for collocation solve": volume matrices G_j, the
upwind face matrix F_d, mass matrices), for the degree-1 tensor element.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this module.  The HIP library never
uses it and shares no code with it.

Written to be read against the weak form: for every cell K and every bilinear
test function v on K,

    - int_K (Omega . grad v) psi  +  sum over faces f of K with Omega.n > 0 of
      int_f (Omega.n) psi v  +  int_K sigma_t psi v
  =   int_K s v  +  sum over faces with Omega.n < 0 of int_f |Omega.n| psi_up v

where psi_up is the trace of the upwind neighbour (or the inflow data on the
domain boundary).  The paper's face matrix (central flux plus half the jump
penalty) equals this upwind flux.  Each cell's 4 x 4 system is solved with a
library solve, cells visited in upwind order.

Discrete objects (all plain numpy, float64):
  * cell e = j*nx + i on [x0, x0 + nx hx] x [y0, y0 + ny hy];
  * nodal basis at the cell corners, local node a = ix + 2*iy (ix = 0 left,
    1 right; iy = 0 bottom, 1 top);
  * source s given by its nodal values per cell (the Q1 interpolant), so the
    right-hand side is M s;
  * inflow data per inflow-face node: inflow_x[d, j, iy] is the value at node iy
    of row j's x-inflow face (the left face when mu > 0, the right face
    otherwise); inflow_y[d, i, ix] likewise on column i's y-inflow face.
"""
from __future__ import annotations

import numpy as np

# 1D element matrices on [0, 1] with N0 = 1 - xi, N1 = xi
_M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])   # int N_i N_j
_D1 = np.array([[-0.5, -0.5], [0.5, 0.5]])                          # int N_i' N_j
_E0 = np.array([[1.0, 0.0], [0.0, 0.0]])                            # N_i(0) N_j(0)
_E1 = np.array([[0.0, 0.0], [0.0, 1.0]])                            # N_i(1) N_j(1)


def _tensor(ax, ay):
    """4 x 4 matrix with entry [a][b] = ax[ia][ib] * ay[ja][jb], a = ia + 2 ja."""
    out = np.empty((4, 4))
    for a in range(4):
        for b in range(4):
            out[a, b] = ax[a % 2, b % 2] * ay[a // 2, b // 2]
    return out


def element_matrices(hx, hy):
    """Mass M, volume G_x = int dv/dx u, G_y, and the four face mass matrices."""
    return {
        "M": hx * hy * _tensor(_M1, _M1),
        "Gx": hy * _tensor(_D1, _M1),
        "Gy": hx * _tensor(_M1, _D1),
        "left": hy * _tensor(_E0, _M1),
        "right": hy * _tensor(_E1, _M1),
        "bottom": hx * _tensor(_M1, _E0),
        "top": hx * _tensor(_M1, _E1),
    }


def local_matrix(em, mu, eta, sigt):
    """Left-hand side of one cell and direction (upwind: outflow faces on the matrix)."""
    out_x = em["right"] if mu > 0 else em["left"]
    out_y = em["top"] if eta > 0 else em["bottom"]
    return -mu * em["Gx"] - eta * em["Gy"] + abs(mu) * out_x + abs(eta) * out_y + sigt * em["M"]


def sweep(nx, ny, hx, hy, mu, eta, sigma_t, src, inflow_x, inflow_y):
    """Q1 upwind DG solve for each direction.

    mu, eta [nd]; sigma_t [ny*nx]; src [nd, ny*nx, 4] nodal source values;
    inflow_x [nd, ny, 2]; inflow_y [nd, nx, 2]  ->  psi [nd, ny*nx, 4]."""
    em = element_matrices(hx, hy)
    nd = len(mu)
    psi = np.zeros((nd, ny * nx, 4))
    for d in range(nd):
        m, e = float(mu[d]), float(eta[d])
        in_x = em["left"] if m > 0 else em["right"]
        in_y = em["bottom"] if e > 0 else em["top"]
        irange = range(nx) if m > 0 else range(nx - 1, -1, -1)
        jrange = range(ny) if e > 0 else range(ny - 1, -1, -1)
        for j in jrange:
            for i in irange:
                c = j * nx + i
                A = local_matrix(em, m, e, float(sigma_t[c]))
                # upwind traces on the two inflow faces, as nodal vectors of this cell
                up = np.zeros(4)
                iu = i - 1 if m > 0 else i + 1
                face_ix = 0 if m > 0 else 1          # this cell's nodes on the x-inflow face
                for iy in range(2):
                    a = face_ix + 2 * iy
                    if 0 <= iu < nx:
                        up[a] = psi[d, j * nx + iu, (1 - face_ix) + 2 * iy]
                    else:
                        up[a] = inflow_x[d, j, iy]
                rhs = em["M"] @ src[d, c] + abs(m) * (in_x @ up)
                up = np.zeros(4)
                ju = j - 1 if e > 0 else j + 1
                face_iy = 0 if e > 0 else 1
                for ix in range(2):
                    a = ix + 2 * face_iy
                    if 0 <= ju < ny:
                        up[a] = psi[d, ju * nx + i, ix + 2 * (1 - face_iy)]
                    else:
                        up[a] = inflow_y[d, i, ix]
                rhs = rhs + abs(e) * (in_y @ up)
                psi[d, c] = np.linalg.solve(A, rhs)
    return psi


def node_coordinates(nx, ny, hx, hy, x0=0.0, y0=0.0):
    """Physical coordinates of the four nodes of every cell: [ny*nx, 4, 2]."""
    xy = np.empty((ny * nx, 4, 2))
    for j in range(ny):
        for i in range(nx):
            for a in range(4):
                xy[j * nx + i, a, 0] = x0 + (i + a % 2) * hx
                xy[j * nx + i, a, 1] = y0 + (j + a // 2) * hy
    return xy


def boundary_balance(nx, ny, hx, hy, mu, eta, sigma_t, src, inflow_x, inflow_y, psi):
    """Per direction: (absorption + outflow through the domain boundary) minus (source +
    inflow through the domain boundary), all from the discrete solution (test function 1)."""
    em = element_matrices(hx, hy)
    ones = np.ones(4)
    res = np.zeros(len(mu))
    for d in range(len(mu)):
        m, e = float(mu[d]), float(eta[d])
        total = 0.0
        for c in range(nx * ny):
            total += sigma_t[c] * ones @ em["M"] @ psi[d, c] - ones @ em["M"] @ src[d, c]
        # outflow faces on the boundary
        io = nx - 1 if m > 0 else 0
        fo = em["right"] if m > 0 else em["left"]
        fi = em["left"] if m > 0 else em["right"]
        face_ix = 0 if m > 0 else 1
        for j in range(ny):
            total += abs(m) * ones @ fo @ psi[d, j * nx + io]
            up = np.zeros(4)
            for iy in range(2):
                up[face_ix + 2 * iy] = inflow_x[d, j, iy]
            total -= abs(m) * ones @ fi @ up
        jo = ny - 1 if e > 0 else 0
        fo = em["top"] if e > 0 else em["bottom"]
        fi = em["bottom"] if e > 0 else em["top"]
        face_iy = 0 if e > 0 else 1
        for i in range(nx):
            total += abs(e) * ones @ fo @ psi[d, jo * nx + i]
            up = np.zeros(4)
            for ix in range(2):
                up[ix + 2 * face_iy] = inflow_y[d, i, ix]
            total -= abs(e) * ones @ fi @ up
        res[d] = total
    return res
