"""GPU: the launch-shape autotuner picks a valid configuration, the chosen
configuration computes the same forces as the default one, and the choice is
cached and reused."""
import numpy as np
import pytest

import md_inputs

pytestmark = pytest.mark.gpu


def test_autotune_picks_and_caches(tmp_path):
    from paper_2109_10876_amd import MDSystem, autotune
    print("case: autotune", flush=True)
    cfg = md_inputs.lj_fluid(12, temperature=1.0, seed=29, jitter_amp=0.05)

    def make(mode, tile_cells, tile_rows=(1, 1)):
        return MDSystem(cfg.natoms, cfg.box, cfg.pos, cfg.vel, rc=cfg.rc, skin=cfg.skin,
                        dt=cfg.dt, mode=mode, tile_cells=tile_cells, tile_rows=tile_rows)

    cache = str(tmp_path / "tune.json")
    key = autotune.signature(cfg.natoms, cfg.box, cfg.rc, cfg.skin, 1)
    best, trials = autotune.tune(make, key, steps=4, warmup=2, cache=cache)
    assert best["mode"] in ("full", "tile")
    assert len(trials) >= 5 and all(ms > 0 for _, ms in trials)
    again, trials2 = autotune.tune(make, key, steps=4, warmup=2, cache=cache)
    assert again == best and len(trials2) == len(trials)
    autotune.apply(best)
    a = make(best["mode"], best.get("tile_cells"), tuple(best.get("tile_rows", (1, 1))))
    a.setup()
    a.ensure_list()
    autotune.apply({"mode": "full", "batch": 4, "tile_threads": 256})
    b = make("full", None)
    b.setup()
    b.ensure_list()
    assert np.abs(a.forces_np() - b.forces_np()).max() < 1e-10
