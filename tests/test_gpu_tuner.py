"""Sweep launch-shape tuner (dlr_sweep_shape / dlr_set_sweep_shape): the launch shape of the
transport sweeps changes no arithmetic, so every candidate shape -- down to a single persistent
workgroup -- gives bitwise the same steps; the tuner's choice is one of the candidates and is kept
for the next instance with the same grid, directions and precision."""
import numpy as np
import pytest

from synth import problems

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_every_sweep_shape_gives_the_same_steps(prec):
    from paper_2601_18705_amd import dlrtrt
    p = problems.random_medium(n=96, n_polar=4, n_azim=8, rank=8, dt=0.005, nsteps=2, seed=5)
    p["ny"] = 77   # ragged columns
    m = 96 * 77
    for key in ("sigma_a", "rho_cv", "T_init"):
        p[key] = p[key][:m]
    if p.get("q_ext") is not None:
        p["q_ext"] = p["q_ext"][:m]
    p["precision"] = prec
    p["si_tol"] = 1e-6 if prec else 1e-13
    shapes = [(4, 512), (2, 256), (2, 1), (4, 3), (4, 1024)] + ([(8, 1024), (8, 2)] if prec else [])
    ref = None
    for sh in shapes:
        with dlrtrt.Instance(p) as inst:
            inst.set_sweep_shape(*sh)
            inst.step(2)
            assert inst.sweep_shape() == sh
            E, T = inst.read_fields()
        print(f"[tuner] precision {prec} shape {sh} done", flush=True)
        if ref is None:
            ref = (E, T)
        else:
            assert np.array_equal(E, ref[0]) and np.array_equal(T, ref[1]), f"shape {sh}"
    with dlrtrt.Instance(p) as inst:
        assert inst.sweep_shape() == (0, 0)
        inst.step(2)
        tuned = inst.sweep_shape()
        E, T = inst.read_fields()
    print(f"[tuner] precision {prec}: tuned shape {tuned}", flush=True)
    assert tuned[0] in ((2, 4, 8) if prec else (2, 4)) and tuned[1] in (256, 512, 1024)
    assert np.array_equal(E, ref[0]) and np.array_equal(T, ref[1])
    with dlrtrt.Instance(p) as inst:
        inst.step(1)
        assert inst.sweep_shape() == tuned      # kept for the same grid, directions and precision


def test_sweep_shape_arguments():
    from paper_2601_18705_amd import dlrtrt
    p = problems.random_medium(n=32, n_polar=2, n_azim=8, rank=4, dt=0.005, nsteps=1, seed=2)
    p["precision"] = 0
    with dlrtrt.Instance(p) as inst:
        for bad in [(3, 512), (8, 512), (4, 0), (4, 70000), (0, 5)]:
            with pytest.raises(dlrtrt.DlrError):
                inst.set_sweep_shape(*bad)
        inst.set_sweep_shape(0, 0)


def test_deep_prefetch_on_short_columns():
    """Eight chunks in flight on columns shorter than eight chunks (ny < 50): the head of the
    chunk loop stops at the last chunk; the step equals the default shape's bitwise."""
    from paper_2601_18705_amd import dlrtrt
    out = []
    for sh in [(4, 512), (8, 512), (8, 1)]:
        p = problems.random_medium(n=40, n_polar=2, n_azim=8, rank=6, dt=0.005, nsteps=2, seed=9)
        p["ny"] = 21
        m = 40 * 21
        for key in ("sigma_a", "rho_cv", "T_init"):
            p[key] = p[key][:m]
        if p.get("q_ext") is not None:
            p["q_ext"] = p["q_ext"][:m]
        p["precision"] = 1
        with dlrtrt.Instance(p) as inst:
            inst.set_sweep_shape(*sh)
            inst.step(2)
            out.append(inst.read_fields())
    for E, T in out[1:]:
        assert np.array_equal(E, out[0][0]) and np.array_equal(T, out[0][1])
