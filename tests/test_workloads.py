"""The seeded input generator: deterministic, tile-ordered, in range."""
import numpy as np

import pic_workloads as pw


def test_species_state_layout_and_determinism():
    spec = pw.SpeciesSpec(-1.0, (4, 2), (0.1, 0.2, 0.3), (0.5, 0.0, -0.1))
    a = pw.species_state(32, 16, 8, spec, seed=9)
    b = pw.species_state(32, 16, 8, spec, seed=9)
    for k in a:
        assert np.array_equal(a[k], b[k])
    n = 32 * 16 * 8
    assert a["ix"].size == n and a["ix"].dtype == np.int32 and a["ux"].dtype == np.float32
    assert (a["x"] >= 0).all() and (a["x"] < 1).all() and (a["y"] >= 0).all() and (a["y"] < 1).all()
    tile = (a["iy"] // 8) * 4 + a["ix"] // 8
    assert (np.diff(tile) >= 0).all()                          # tile order
    assert np.bincount(tile).tolist() == [8 * 8 * 8] * 8       # equal tiles
    cells = a["iy"] * 32 + a["ix"]
    assert np.bincount(cells).tolist() == [8] * (32 * 16)      # 8 per cell
    assert np.all(cells[:64] != cells[1:65])                  # neighbours in different cells
    for k, name in enumerate(("ux", "uy", "uz")):
        v = a[name].astype(np.float64)
        assert abs(v.mean() - spec.u_fl[k]) < 5 * spec.u_th[k] / np.sqrt(n)
        assert abs(v.std() / spec.u_th[k] - 1) < 0.05
    c = pw.species_state(32, 16, 8, spec, seed=10)
    assert not np.array_equal(a["ux"], c["ux"])


def test_cell_box_makes_empty_tiles():
    spec = pw.SpeciesSpec(-1.0, (2, 2))
    a = pw.species_state(32, 32, 8, spec, seed=1, cell_box=(0, 12, 4, 20))
    assert a["ix"].max() < 12 and a["iy"].min() >= 4 and a["iy"].max() < 20
    tile = (a["iy"] // 8) * 4 + a["ix"] // 8
    assert (np.diff(tile) >= 0).all()
