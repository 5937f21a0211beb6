"""The offline FOM reference writer: its parameter sets are the benchmark's draws (held-out
parameters, optionally the ones the uneven batch assigns to one model) and its states are the
monolithic FOM Newton solutions of those parameters."""
import numpy as np

import seeded_inputs as si
from oracle import fom_reference as fr
from oracle.burgers import BurgersFOM, Grid, solve_fom


def test_sets_follow_the_benchmark_draws(tmp_path):
    out = str(tmp_path / "ref.npz")
    assert fr.main(["--grid", "6", "5", "--set", "held:3:10:4", "--set", "part:2:12:3:1/3",
                    "--workers", "1", "--out", out]) == 0
    ref = np.load(out)
    assert np.array_equal(ref["held_mu"], si.heldout_mu(10, 3)[:4])
    want = si.heldout_mu(12, 2)[si.model_assignment(12, 3, 2) == 1][:3]
    assert ref["part_mu"].shape == (3, 2) and np.array_equal(ref["part_mu"], want)
    assert tuple(ref["grid"]) == (6, 5)
    # each stored state is the FOM solution of its parameter (rounded to FP32)
    fom = BurgersFOM(Grid(6, 5))
    for name in ("held", "part"):
        for mu, x in zip(ref[f"{name}_mu"], ref[f"{name}_x"]):
            r = solve_fom(fom, tuple(mu))
            assert r.converged
            assert np.max(np.abs(x - r.x)) <= 1e-6 * np.max(np.abs(r.x))
