"""GPU parity of the augmented-basis step (dlr_create_augmented) against the oracle's
dlr_step with p["augment"] set: the swept columns and the old basis span a 2r-column
Galerkin space, and the SVD result is truncated back to rank r.

The comparison follows the plain parity tests: E_r and T (relative L2, max-norm and
per-cell T) and the energy sum, outflow and inflow at every step, FP64 to 1e-10 and
FP32 sweeps to 1e-4; DEIM picks compared first, a differing pick allowed only at an
oracle decision edge within what the precision can perturb, and then the oracle's
picks are replayed.  A truncation cuts the spectrum between sigma_r and sigma_{r+1},
so the uncertainty of the kept angular columns is judged from the gaps among all 2r
singular values of the previous step (the oracle's sigma_all), not the r kept ones.
"""
import numpy as np
import pytest

from oracle import dlr_oracle as O
from synth import problems

from _parity import check_balance, check_fields, divergence_allowed, rel

pytestmark = pytest.mark.gpu

FP32 = {"precision": 1, "si_tol": 1e-6}


def augmented(p):
    q = dict(p)
    q["augment"] = True
    return q


def oracle_run(p, nsteps):
    _, ref = O.run_dlr(augmented(p), nsteps=nsteps)
    return ref


def gpu_run(p, nsteps, forced=None, factors=False):
    from paper_2601_18705_amd import dlrtrt
    out = []
    with dlrtrt.Instance(p, method="augmented") as inst:
        for n in range(nsteps):
            if forced is not None:
                inst.force_selection(forced[n])
            inst.step(1)
            E, T = inst.read_fields()
            X, S, W, sel = inst.read_factors()
            rec = {"E_r": E, "T": T, "sel": sel.copy(), "stats": inst.read_stats()}
            if factors:
                rec.update(X=X, S=S, W=W)
            out.append(rec)
    return out


def compare(p, nsteps, tol, label, gpu_overrides=None, ref=None, factors=False):
    pg = dict(p, **(gpu_overrides or {}))
    prec = int(pg.get("precision", 0))
    print(f"[augmented] {label}: {p['nx']}x{p['ny']} q{p['n_polar']}x{p['n_azim']} r{p['rank']} "
          f"(Galerkin rank {2 * p['rank']}) prec{prec} steps{nsteps}", flush=True)
    if ref is None:
        ref = oracle_run(p, nsteps)
    g = gpu_run(pg, nsteps, factors=factors)
    same = all(np.array_equal(np.asarray(a["sel"]), np.asarray(b["sel"])) for a, b in zip(g, ref))
    if not same:
        first = next(n for n, (a, b) in enumerate(zip(g, ref)) if not np.array_equal(a["sel"], b["sel"]))
        j = int(np.flatnonzero(np.asarray(g[first]["sel"]) != np.asarray(ref[first]["sel"]))[0])
        spectrum = [dict(h, sigma=h["sigma_all"]) for h in ref]
        ok, edge, limit = divergence_allowed(spectrum, first, j, prec)
        assert ok, (
            f"{label}: DEIM pick {j} differs at step {first} although the oracle's decision edge "
            f"{edge:.3e} is above the allowed {limit:.3e}: "
            f"gpu {g[first]['sel'].tolist()} oracle {ref[first]['sel'].tolist()}")
        print(f"[augmented] {label}: pick {j} differs at step {first} (decision edge {edge:.3e}, "
              f"allowed {limit:.3e}); replaying the oracle's picks", flush=True)
        g = gpu_run(pg, nsteps, forced=[h["sel"] for h in ref], factors=factors)
    worst = 0.0
    for n, (a, b) in enumerate(zip(g, ref)):
        worst = max(worst, check_fields(a["E_r"], a["T"], b, tol, f"{label} step {n}"))
        check_balance(a["stats"], b, tol, f"{label} step {n}")
        assert a["stats"]["rank"] == p["rank"]
    print(f"[augmented] {label}: worst error {worst:.3e} (free-running={same}); "
          f"SI iterations {[a['stats']['si_iters'] for a in g]}", flush=True)
    return g, ref


def test_slab_beam_fp64():
    compare(problems.slab_beam(), 10, 1e-10, "slab_beam fp64")


@pytest.mark.parametrize("nx,ny,npol,naz,rank", [
    (50, 37, 4, 8, 5),       # ragged strip tail, odd rank, Galerkin rank 10
    (130, 20, 4, 8, 12),     # three strips, Galerkin rank 24 (two 16-plane tiles)
    (7, 64, 3, 4, 1),        # single partial strip, rank one
    (33, 29, 4, 8, 16),      # Galerkin rank 32
    (36, 30, 8, 8, 20),      # Galerkin rank 40: the three-tile matrix-core paths, the 8 x 8-block L-step
    (40, 33, 8, 8, 32),      # Galerkin rank 64 = every ordinate: the four-tile paths
])
def test_ragged_shapes_fp64(nx, ny, npol, naz, rank):
    p = problems.slab_beam(nx=nx, n_polar=npol, n_azim=naz, rank=rank, nsteps=4)
    p["ny"] = ny
    n = nx * ny
    rng = np.random.default_rng(nx * 1000 + ny)
    p["sigma_a"] = rng.uniform(0.5, 20.0, n)
    p["rho_cv"] = rng.uniform(0.5, 2.0, n)
    p["T_init"] = rng.uniform(0.01, 0.3, n)
    p["q_ext"] = rng.uniform(0.0, 1.0, n)
    p["bc"] = [1, 1, 0, 1]
    p["T_b"] = [1.0, 0.5, 0.0, 0.8]
    compare(p, 4, 1e-10, f"ragged {nx}x{ny}")


def test_random_medium_fp64_and_fp32():
    p = problems.random_medium(n=128, nsteps=6)
    ref = oracle_run(p, 6)
    compare(p, 6, 1e-10, "random medium 128^2 fp64", ref=ref)
    compare(p, 6, 1e-4, "random medium 128^2 fp32", FP32, ref=ref)


@pytest.mark.parametrize("rank", [12, 20])
def test_bf16_projections(rank):
    """Split-BF16 projection operands (with FP32 sweeps) on the 2r-column basis, whose old-basis rows of
    <X0_i, X_j> are a separate count: within 1e-4 of the FP64 oracle."""
    p = problems.slab_beam(nx=24, n_polar=8, n_azim=8, rank=rank, nsteps=3)
    compare(p, 3, 1e-4, f"slab 24^2 rank {rank} bf16 projections", {"precision": 2, "si_tol": 1e-6})


_FULL = {}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("label,over,tol", [("fp64", None, 1e-10), ("fp32", FP32, 1e-4)])
def test_full_size_random_medium(label, over, tol):
    """The benchmark workload at its full size (1024^2 cells, 32 x 64 ordinates, r = 32: a
    Galerkin rank of 64): four steps against the oracle."""
    p = problems.random_medium(nsteps=4)
    if "ref" not in _FULL:
        _FULL["ref"] = oracle_run(p, 4)
    compare(p, 4, tol, f"random medium 1024^2 {label}", over, ref=_FULL["ref"])


def test_truncated_factors_match_the_oracle():
    """The truncated state itself: X orthonormal, S diagonal to rounding with the oracle's r
    largest singular values, and X S W^T equal to the oracle's on every cell and ordinate."""
    p = problems.slab_beam(nx=24, n_polar=4, n_azim=8, rank=6, nsteps=4)
    quad = O.quadrature(4, 8)
    grid = O.grid_of(p)
    pa = augmented(p)
    st = O.dlr_initial_state(pa, quad)
    refs = []
    for _ in range(4):
        st, stats = O.dlr_step(pa, quad, st)
        refs.append((st.X @ st.S @ st.W.T, stats["sigma"]))
    g = gpu_run(p, 4, factors=True)
    for n, (a, (psi_ref, sig_ref)) in enumerate(zip(g, refs)):
        X, S, W = a["X"], a["S"], a["W"]
        assert np.max(np.abs(grid.area * X.T @ X - np.eye(6))) < 1e-12, n
        assert np.max(np.abs(W.T @ (quad.w[:, None] * W) - np.eye(6))) < 1e-12, n
        d = np.diag(S)
        assert np.max(np.abs(S - np.diag(d))) <= 1e-13 * d[0], n
        assert np.max(np.abs(d - sig_ref)) <= 1e-10 * sig_ref[0], (n, d, sig_ref)
        # the rows of X are in the library's cell order (j * nx + i), as the oracle's
        assert rel(X @ S @ W.T, psi_ref) < 1e-10, n


@pytest.mark.parametrize("uniform", [True, False])
def test_initial_basis_is_the_oracles_completion(uniform):
    """The rank-one initial state's spatial basis, completed by the graded monomials: Cholesky QR of
    [B(T_init), monomials] on the device (the constant left out when B(T_init) is constant) against the
    oracle's CGS2 of [B(T_init), 0, ...]."""
    from paper_2601_18705_amd import dlrtrt
    p = problems.slab_beam(nx=30, n_polar=4, n_azim=8, rank=9, nsteps=1)
    p["ny"] = 21
    n = 30 * 21
    p["sigma_a"], p["rho_cv"], p["q_ext"] = np.ones(n), np.ones(n), np.zeros(n)
    if not uniform:
        rng = np.random.default_rng(5)
        p["T_init"] = rng.uniform(0.2, 0.9, n)
    else:
        p["T_init"] = np.full(n, 0.4)
    quad = O.quadrature(4, 8)
    ref = O.dlr_initial_state(augmented(p), quad)
    with dlrtrt.Instance(p, method="augmented") as inst:
        X, S, W, _ = inst.read_factors()
    assert np.max(np.abs(X - ref.X)) < 1e-11 * np.max(np.abs(ref.X))
    assert np.max(np.abs(S - ref.S)) < 1e-12 * abs(ref.S[0, 0])


def test_checkpoint_resume():
    from paper_2601_18705_amd import dlrtrt
    p = problems.slab_beam(nx=40, n_polar=4, n_azim=8, rank=6, nsteps=6)
    ref = gpu_run(p, 6)
    with dlrtrt.Instance(p, method="augmented") as a:
        a.step(3)
        X, S, W, _ = a.read_factors()
        _, T = a.read_fields()
    with dlrtrt.Instance(p, method="augmented") as b:
        b.load_factors(X, S, W, T)
        b.step(3)
        E2, T2 = b.read_fields()
    assert rel(E2, ref[-1]["E_r"]) < 1e-12 and rel(T2, ref[-1]["T"]) < 1e-12


def test_runs_are_bitwise_reproducible():
    p = problems.checkerboard(n=96, n_polar=4, n_azim=8, rank=6, nsteps=3)
    a = gpu_run(p, 3)
    b = gpu_run(p, 3)
    for x, y in zip(a, b):
        assert np.array_equal(x["E_r"], y["E_r"]) and np.array_equal(x["T"], y["T"])


def test_with_dsa_on_a_thick_checkerboard():
    """The augmented step under diffusion synthetic acceleration (sigma = 10^4 in alternating blocks,
    hot start): the accelerated source iteration reaches the oracle's fixed point, FP64 to 1e-10."""
    p = problems.checkerboard(n=28, n_polar=4, n_azim=8, rank=6, nsteps=2)
    p["sigma_a"] = problems.checkerboard_sigma(p, thick=1e4, thin=1.0)
    p["T_init"] = np.full(p["nx"] * p["ny"], 1.0)
    p["si_tol"] = 1e-13
    p["dsa"] = 1
    g, ref = compare(p, 2, 1e-10, "thick checkerboard with DSA")
    assert max(a["stats"]["si_iters"] for a in g) <= 8


def test_equilibrium_stays_put_through_the_fallbacks():
    """T_init = T_b on all four sides and no source: psi stays B(T) everywhere.  The swept columns are
    then all alike, the completion monomials fill both bases, and the 2r Cholesky QR meets exactly
    dependent columns, so the CGS2 fallbacks run; the truncated state has a single nonzero singular
    value (its other factors are arbitrary, so the DEIM picks are not compared).  The fields hold the
    closed form, and the energy tallies equal the oracle's."""
    from paper_2601_18705_amd import dlrtrt
    p = problems.slab_beam(nx=20, n_polar=4, n_azim=8, rank=5, nsteps=3)
    n = p["nx"] * p["ny"]
    p["T_init"] = np.full(n, 0.5)
    p["bc"] = [1, 1, 1, 1]
    p["T_b"] = [0.5] * 4
    ref = oracle_run(p, 3)
    with dlrtrt.Instance(p, method="augmented") as inst:
        for n_, b in enumerate(ref):
            inst.step(1)
            E, T = inst.read_fields()
            st = inst.read_stats()
            assert np.max(np.abs(T - 0.5)) < 1e-13, n_
            assert np.max(np.abs(E - 0.5 ** 4)) < 1e-13 * 0.5 ** 4, n_
            check_balance(st, b, 1e-12, f"equilibrium step {n_}")


def test_rank_limit_is_rejected():
    from paper_2601_18705_amd import dlrtrt
    for p in (problems.slab_beam(nx=16, n_polar=2, n_azim=4, rank=5, nsteps=1),    # 2 r > 8 ordinates
              problems.slab_beam(nx=16, n_polar=8, n_azim=8, rank=33, nsteps=1),   # 2 r > 64
              problems.slab_beam(nx=3, n_polar=4, n_azim=8, rank=5, nsteps=1)):    # 2 r > 9 cells
        with pytest.raises(dlrtrt.DlrError) as ei:
            dlrtrt.Instance(p, method="augmented")
        assert ei.value.status == -1
