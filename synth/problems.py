"""Seeded synthetic problem generator for gray thermal radiative transfer on 2D
structured meshes.

This module only builds *inputs*: grid extents, material fields, boundary
conditions and solver knobs.  It contains none of the method's arithmetic
(no quadrature, no linearisation, no sweeps, no factorisations), so both the
FP64 CPU oracle and the HIP library consume the same arrays without sharing
any code of the method.

Field conventions (shared by every consumer):
  * cells are numbered e = j*nx + i (i along x, j along y), arrays are float64
    of length ny*nx;
  * ``sigma_a``  absorption opacity sigma(T0) (opacity is held fixed in time);
  * ``rho_cv``   volumetric heat capacity rho*c_v;
  * ``q_ext``    external isotropic radiation source, integrated over angle
                 (the per-steradian source is q_ext / (4 pi));
  * ``T_init``   initial material temperature; the initial radiation field is
                 the isotropic Planck intensity of T_init;
  * ``bc``       boundary kind per side (left, right, bottom, top):
                 0 = vacuum, 1 = isotropic inflow at temperature T_b, 2 = reflecting;
  * ``T_b``      inflow temperature per side (used when bc == 1).

The five named workloads follow the configurations the method is measured on:
a small homogeneous slab with a left-edge beam, a 7x7 two-opacity checkerboard
with a central source, a large log-normal random medium, a batch of uneven
random-medium instances, and a Poisson request stream.
"""
from __future__ import annotations

import numpy as np

BC_VACUUM = 0
BC_INFLOW = 1
BC_REFLECT = 2

PREC_FP64 = 0          # every phase in FP64
PREC_FP32_SWEEP = 1    # FP32 sweeps and projections, FP64 elsewhere
PREC_FP32_SWEEP_BF16 = 2  # FP32 sweeps, BF16 projections with FP32 accumulation


def base_problem(nx, ny, extent=(0.0, 1.0, 0.0, 1.0), n_polar=8, n_azim=8, rank=8,
                 dt=0.01, c=1.0, a=1.0, nsteps=10):
    """A homogeneous problem skeleton (sigma_a = 1, rho_cv = 1, cold start, vacuum)."""
    n = nx * ny
    return dict(
        nx=int(nx), ny=int(ny),
        x0=float(extent[0]), x1=float(extent[1]), y0=float(extent[2]), y1=float(extent[3]),
        n_polar=int(n_polar), n_azim=int(n_azim), rank=int(rank),
        dt=float(dt), c=float(c), a=float(a), nsteps=int(nsteps),
        sigma_a=np.ones(n), rho_cv=np.ones(n), q_ext=np.zeros(n),
        T_init=np.full(n, 1e-3),
        bc=[BC_VACUUM] * 4, T_b=[0.0] * 4,
        precision=PREC_FP64, si_tol=1e-14, si_max_iter=10000, deim_tie_tol=1e-6,
    )


def cell_centres(p):
    """Cell-centre coordinates (xc[ny*nx], yc[ny*nx]) in the e = j*nx + i order."""
    hx = (p["x1"] - p["x0"]) / p["nx"]
    hy = (p["y1"] - p["y0"]) / p["ny"]
    xc = p["x0"] + (np.arange(p["nx"]) + 0.5) * hx
    yc = p["y0"] + (np.arange(p["ny"]) + 0.5) * hy
    X, Y = np.meshgrid(xc, yc)          # [ny, nx]
    return X.ravel(), Y.ravel()


def gaussian_random_field(n, corr_cells, seed):
    """Periodic stationary Gaussian field on an n x n grid by spectral synthesis.

    Covariance exp(-d^2 / (2 l^2)) with l = corr_cells (in cells); the sample is
    shifted and scaled to mean 0 and variance 1.  Seeded with numpy's PCG64.
    """
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n))
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    kx, ky = np.meshgrid(k, k)
    amp = np.exp(-0.25 * corr_cells ** 2 * (kx ** 2 + ky ** 2))   # sqrt of the spectral density
    g = np.real(np.fft.ifft2(np.fft.fft2(white) * amp))
    g -= g.mean()
    g /= g.std()
    return g.ravel()


def lognormal_sigma(n, seed, mu=0.0, s=1.5, corr_cells=16):
    return np.exp(mu + s * gaussian_random_field(n, corr_cells, seed))


def checkerboard_sigma(p, thick=100.0, thin=1.0):
    """Unit blocks of the domain by cell centre; (bx + by) odd -> thick."""
    xc, yc = cell_centres(p)
    bx = np.floor(xc - p["x0"]).astype(np.int64)
    by = np.floor(yc - p["y0"]).astype(np.int64)
    return np.where((bx + by) % 2 == 1, thick, thin).astype(np.float64)


# --------------------------------------------------------------------------- named workloads

def slab_beam(nx=32, n_polar=8, n_azim=8, rank=8, dt=0.01, nsteps=10):
    """32^2 homogeneous unit square, cold start, isotropic inflow at T_b = 1 on the left."""
    p = base_problem(nx, nx, (0.0, 1.0, 0.0, 1.0), n_polar, n_azim, rank, dt, nsteps=nsteps)
    p["bc"] = [BC_INFLOW, BC_VACUUM, BC_VACUUM, BC_VACUUM]
    p["T_b"] = [1.0, 0.0, 0.0, 0.0]
    p["name"] = f"slab_beam_{nx}x{nx}_q{n_polar}x{n_azim}_r{rank}"
    return p


def checkerboard(n=256, n_polar=16, n_azim=32, rank=16, dt=0.005, nsteps=100):
    """7x7 unit-block checkerboard on [0,7]^2 (sigma 100 / 1), unit source in block (3,3)."""
    p = base_problem(n, n, (0.0, 7.0, 0.0, 7.0), n_polar, n_azim, rank, dt, nsteps=nsteps)
    p["sigma_a"] = checkerboard_sigma(p)
    xc, yc = cell_centres(p)
    inside = (xc > 3.0) & (xc < 4.0) & (yc > 3.0) & (yc < 4.0)
    p["q_ext"] = np.where(inside, 1.0, 0.0)
    p["name"] = f"checkerboard_{n}x{n}_q{n_polar}x{n_azim}_r{rank}"
    return p


def random_medium(n=1024, n_polar=32, n_azim=64, rank=32, dt=0.002, nsteps=200, seed=3):
    """Log-normal opacity (s = 1.5, 16-cell correlation), left inflow at T_b = 1."""
    p = base_problem(n, n, (0.0, 1.0, 0.0, 1.0), n_polar, n_azim, rank, dt, nsteps=nsteps)
    p["sigma_a"] = lognormal_sigma(n, seed)
    p["bc"] = [BC_INFLOW, BC_VACUUM, BC_VACUUM, BC_VACUUM]
    p["T_b"] = [1.0, 0.0, 0.0, 0.0]
    p["name"] = f"random_medium_{n}x{n}_q{n_polar}x{n_azim}_r{rank}_seed{seed}"
    return p


def batch_instances(count=256, seed=4, n_polar=16, n_azim=32, dt=0.005, nsteps=50,
                    sizes=(64, 128, 256), ranks=(4, 8, 16, 24)):
    """Independent random-medium instances of uneven grid size and rank."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(rng.choice(sizes))
        r = int(rng.choice(ranks))
        fseed = int(rng.integers(0, 2 ** 31 - 1))
        p = random_medium(n, n_polar, n_azim, r, dt, nsteps, seed=fseed)
        p["name"] = f"batch{k}_{n}x{n}_r{r}"
        out.append(p)
    return out


def request_specs(seed=5, rate_hz=200.0, count=2000, n_polar=16, n_azim=32, dt=0.005,
                  sizes=(64, 128, 256, 512, 1024), ranks=(8, 16, 24, 32), steps=(20, 200), window_s=None):
    """Poisson arrivals of checkerboard or random-medium problems as lazy specs:
    [(t_arrival, build, n_steps, name)], build() returning the problem dict.  Stops after
    `count` requests or at the first arrival past window_s (when given).  The draws do not
    depend on when (or whether) a problem is built."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate_hz)
        if window_s is not None and t > window_s:
            break
        n = int(rng.choice(sizes))
        r = int(rng.choice(ranks))
        ns = int(rng.integers(steps[0], steps[1] + 1))
        board = rng.random() < 0.5
        fseed = int(rng.integers(0, 2 ** 31 - 1))

        def build(n=n, r=r, ns=ns, board=board, fseed=fseed, k=k):
            if board:
                p = checkerboard(n, n_polar, n_azim, r, dt, ns)
            else:
                p = random_medium(n, n_polar, n_azim, r, dt, ns, seed=fseed)
            p["name"] = f"req{k}_{p['name']}"
            return p
        out.append((t, build, ns, f"req{k}"))
    return out


def request_stream(seed=5, rate_hz=200.0, count=2000, **kw):
    """Poisson arrivals of checkerboard or random-medium problems: [(t_arrival, problem)]."""
    return [(t, build()) for t, build, _, _ in request_specs(seed, rate_hz, count, **kw)]


WORKLOADS = {
    "slab_beam": slab_beam,
    "checkerboard": checkerboard,
    "random_medium": random_medium,
}


def q1_sweep_inputs(nx, ny, n_dir, seed, extent=(0.0, 1.0, 0.0, 1.0), sigma_shift=0.0, zero_cells=0.0,
                    dtype=np.float64):
    """Inputs of one bilinear (Q1) DG sweep over n_dir directions.

    Directions: x and y cosines of points drawn uniformly on the unit sphere.
    sigma_t: the log-normal random-medium opacity (s = 1.5, 16-cell correlation,
    cropped from a square field of at least 32 x 32 cells) plus sigma_shift (1 / (c dt) of a time step),
    with a fraction zero_cells of the cells set to exactly zero.  Nodal sources
    [n_dir, ny*nx, 4] and inflow data ([n_dir, ny, 2] on the x-inflow faces,
    [n_dir, nx, 2] on the y-inflow faces) uniform in [0, 1).  Cells e = j*nx + i,
    nodes a = ix + 2*iy."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, n_dir)
    az = rng.uniform(0.0, 2.0 * np.pi, n_dir)
    st = np.sqrt(1.0 - z * z)
    n = max(nx, ny, 32)
    sig = lognormal_sigma(n, seed + 1).reshape(n, n)[:ny, :nx].ravel() + sigma_shift
    if zero_cells > 0.0:
        sig[rng.uniform(0.0, 1.0, sig.size) < zero_cells] = 0.0
    return dict(
        nx=int(nx), ny=int(ny),
        hx=(extent[1] - extent[0]) / nx, hy=(extent[3] - extent[2]) / ny,
        mu=st * np.cos(az), eta=st * np.sin(az),
        sigma_t=sig.astype(dtype),
        src=rng.uniform(0.0, 1.0, (n_dir, nx * ny, 4)).astype(dtype),
        inflow_x=rng.uniform(0.0, 1.0, (n_dir, ny, 2)).astype(dtype),
        inflow_y=rng.uniform(0.0, 1.0, (n_dir, nx, 2)).astype(dtype),
    )
