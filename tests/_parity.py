"""Shared checks of the GPU parity tests: field norms, the energy balance, and the
DEIM near-tie rule that decides when the oracle's picks may be replayed."""
import numpy as np

# A DEIM pick can only change when a perturbation of the residual, relative to its maximum,
# reaches the oracle's decision edge (distance of some |R_q| / max|R| from the tie threshold).
# FP64 paths differ from the oracle by round-off (~1e-13 relative); FP32 sweeps perturb the
# angular basis at ~1e-7, amplified by the elimination.  Below these edges a differing pick
# is a near-tie and the oracle's picks are replayed; above them it fails the test.
NEAR_TIE = {0: 1e-9, 1: 1e-5, 2: 1e-5}


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def maxrel(a, b):
    """max |a - b| / max |b| (the max-norm counterpart of rel)."""
    mb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / mb) if mb > 0 else float(np.max(np.abs(a)))


def check_fields(E, T, ref, tol, where):
    """E_r and T against the oracle: relative L2, max-norm, and per-cell relative T
    (T >= T_init > 0 everywhere, so every cell's temperature is checked on its own scale)."""
    errs = {
        "E_l2": rel(E, ref["E_r"]), "T_l2": rel(T, ref["T"]),
        "E_max": maxrel(E, ref["E_r"]), "T_max": maxrel(T, ref["T"]),
        "T_cell": float(np.max(np.abs(T - ref["T"]) / np.abs(ref["T"]))),
    }
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{where}: " + ", ".join(f"{k} {v:.3e}" for k, v in bad.items()) + f" (tol {tol:g})"
    return max(errs.values())


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
