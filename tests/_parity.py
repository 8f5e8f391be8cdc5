"""Shared checks of the GPU parity tests: field norms, the energy balance, and the
DEIM near-tie rule that decides when the oracle's picks may be replayed."""
import numpy as np

# A DEIM pick can only change when a perturbation of the residual, relative to its maximum,
# reaches the oracle's decision edge (distance of some |R_q| / max|R| from the tie threshold).
# FP64 paths differ from the oracle by round-off (~1e-13 relative); FP32 sweeps perturb the
# angular basis at ~1e-7, amplified by the elimination.  Below these edges a differing pick
# is a near-tie and the oracle's picks are replayed; above them it fails the test.
NEAR_TIE = {0: 1e-9, 1: 1e-5, 2: 1e-5}

# Relative size of the GPU path's perturbation of the coupling matrix S against the oracle's.
PERTURB = {0: 1e-13, 1: 1e-6, 2: 1e-6}


def pick_uncertainty(prev_sigma, prec, j):
    """How far the residual of DEIM pick j may move, relative to its maximum, because the angular
    basis itself is not fixed by the previous step's SVD: a column k of W is determined only up to
    rotations with the columns of nearby singular values, by about eps sigma_0 / gap_k (gap_k: distance
    of sigma_k to the nearest other singular value), and pick j depends on columns 0..j.  Returns 0 at
    the first step (the initial basis comes from the deterministic completion, not from an SVD)."""
    if prev_sigma is None:
        return 0.0
    s = np.abs(np.asarray(prev_sigma, dtype=float))
    r = len(s)
    worst = 0.0
    for k in range(min(j + 1, r)):
        gap = min((abs(s[k] - s[l]) for l in range(r) if l != k), default=s[0])
        worst = max(worst, PERTURB[prec] * s[0] / max(gap, 1e-300))
    return min(worst, 1.0)


def divergence_allowed(ref, step, j, prec):
    """A GPU pick that differs from the oracle's at step `step`, position j, is allowed (and the
    oracle's picks are then replayed) when the oracle's decision edge for that pick is within the
    near-tie level of the precision or within a hundred times the pick's uncertainty from an
    ill-determined angular basis (near-degenerate singular values of the previous step)."""
    edge = float(np.asarray(ref[step]["deim_edge"])[j])
    prev = ref[step - 1]["sigma"] if step > 0 else None
    limit = max(NEAR_TIE[prec], 100.0 * pick_uncertainty(prev, prec, j))
    return edge <= limit, edge, limit


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def maxrel(a, b):
    """max |a - b| / max |b| (the max-norm counterpart of rel)."""
    mb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / mb) if mb > 0 else float(np.max(np.abs(a)))


def check_fields(E, T, ref, tol, where, cell_tol=None):
    """E_r and T against the oracle: relative L2, max-norm, and per-cell relative T
    (T >= T_init > 0 everywhere, so every cell's temperature is checked on its own scale,
    against cell_tol, default tol)."""
    errs = {
        "E_l2": rel(E, ref["E_r"]), "T_l2": rel(T, ref["T"]),
        "E_max": maxrel(E, ref["E_r"]), "T_max": maxrel(T, ref["T"]),
        "T_cell": float(np.max(np.abs(T - ref["T"]) / np.abs(ref["T"]))),
    }
    lim = {k: (tol if k != "T_cell" or cell_tol is None else cell_tol) for k in errs}
    bad = {k: v for k, v in errs.items() if not v <= lim[k]}
    assert not bad, f"{where}: " + ", ".join(f"{k} {v:.3e} (tol {lim[k]:g})" for k, v in bad.items())
    return max(v for k, v in errs.items() if lim[k] == tol)


def check_balance(stats, ref, tol, where):
    """The GPU's energy sum, outflow, inflow and source power against the oracle's."""
    for key, mine, theirs in (("energy", stats["energy"], ref["energy"]),
                              ("outflow", stats["outflow"], ref["outflow"]),
                              ("inflow", stats["inflow"], ref["inflow"])):
        scale = max(abs(theirs), 1e-300)
        if theirs == 0.0:
            assert mine == 0.0, f"{where}: {key} {mine:.6e} vs 0"
        else:
            assert abs(mine - theirs) <= tol * scale, f"{where}: {key} {mine:.15e} vs {theirs:.15e}"


def balance_residual(prev_energy, stats, dt):
    """|E(n+1) - E(n) - dt (source + inflow - outflow)| / E(n+1)."""
    d = stats["energy"] - prev_energy - dt * (stats["source"] + stats["inflow"] - stats["outflow"])
    return abs(d) / abs(stats["energy"])
