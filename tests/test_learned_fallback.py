"""Without a trained network file the learned initialisation leaves the
heuristic parameters untouched (the paper's initialisation is the
fallback); the shipped model file loads without executing anything."""
import os

import numpy as np

from paper_2510_01119_amd import learned_init as LI


def test_missing_model_keeps_heuristic(tmp_path):
    p = np.arange(40, dtype=np.float32).reshape(20, 2)
    out = LI.apply(p, pruned=None, path=str(tmp_path / "absent.npz"))
    assert out is p and np.array_equal(out, np.arange(40, dtype=np.float32).reshape(20, 2))


def test_model_file_round_trip(tmp_path):
    m = LI.InitModel(np.arange(16), np.ones(16), LI.init_master(3), {"note": "x"})
    path = str(tmp_path / "m.npz")
    m.save(path)
    m2 = LI.InitModel.load(path)
    assert np.array_equal(m2.master, m.master) and m2.meta == {"note": "x"}
    assert np.array_equal(m2.shift, m.shift) and np.array_equal(m2.scale, m.scale)


def test_fold_output_is_affine_in_last_layer():
    rng = np.random.default_rng(0)
    master = rng.standard_normal(LI.N_PARAMS).astype(np.float32)
    shift, scale = np.array([1.0, -2.0, 0.5, 3.0]), np.array([2.0, 0.5, 1.5, 0.25])
    f = LI.fold_output(master, shift, scale)
    assert np.array_equal(f[:9408], master[:9408])
    W4, b4 = master[9408:9664].reshape(4, 64).astype(np.float64), master[9664:].astype(np.float64)
    h = rng.standard_normal(64)
    y = W4 @ h + b4
    W4f, b4f = f[9408:9664].reshape(4, 64).astype(np.float64), f[9664:].astype(np.float64)
    assert np.allclose(W4f @ h + b4f, scale * y + shift, rtol=1e-5, atol=1e-5)


def test_shipped_model_loads():
    if not os.path.exists(LI.MODEL_PATH):
        return
    m = LI.InitModel.load()
    assert m.master.shape == (LI.N_PARAMS,) and np.all(np.isfinite(m.master))
