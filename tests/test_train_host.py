"""Host logic of the training loop (no GPU): Adam's row layout and rates per
parameter form, and the conversion of an identity-rotor, tied-scale set to
the isotropic, motion-aware form."""
import numpy as np
import torch

from paper_2510_01119_amd import gs4d as G
from paper_2510_01119_amd.train import ISO_ROWS, LR_DEFAULTS, ROTOR_ROWS, adam_config, to_iso


def test_adam_rows_per_form():
    rot = adam_config(5000)
    iso = adam_config(5000, iso=True)
    assert rot.rows == G.N_FIELDS == len(ROTOR_ROWS)
    assert iso.rows == G.ISO_FIELDS == len(ISO_ROWS)
    for cfg, rows in ((rot, ROTOR_ROWS), (iso, ISO_ROWS)):
        for k, name in enumerate(rows):
            assert np.isclose(cfg.lr0[k], LR_DEFAULTS[name][0])
            assert np.isclose(cfg.lr1[k], LR_DEFAULTS[name][1])
    # isotropic layout: mean xyz t, log s, log s_t, velocity, opacity, rgb
    assert ISO_ROWS[4:6] == ["log_scale"] * 2 and ISO_ROWS[6:9] == ["velocity"] * 3
    frozen = adam_config(100, lrs={"velocity": (0.0, 0.0)}, iso=True)
    assert all(frozen.lr0[k] == 0.0 and frozen.lr1[k] == 0.0 for k in range(6, 9))


def test_to_iso_takes_the_tied_rows():
    n = 5
    p = torch.zeros((G.N_FIELDS, n))
    p[0:4] = torch.arange(4 * n, dtype=torch.float32).reshape(4, n)
    p[4:7] = -4.0
    p[7] = -1.5
    p[8] = 1.0
    p[12] = 1.0
    p[16] = 0.3
    p[17:20] = 0.25
    q = to_iso(p)
    assert q.shape == (G.ISO_FIELDS, n)
    assert torch.equal(q[0:4], p[0:4])
    assert torch.all(q[4] == -4.0) and torch.all(q[5] == -1.5)
    assert torch.all(q[6:9] == 0.0)
    assert torch.all(q[9] == 0.3) and torch.all(q[10:13] == 0.25)


def test_stated_constants():
    """The constants the paper states (Sec. 4.1): position learning rate 1e-5;
    Lite prunes static and dynamic points with lambda 4, Full static points
    with lambda 1 and dynamic points not at all; both take the motion class
    from the Otsu split and adaptive voxels."""
    from paper_2510_01119_amd.scene import PRESETS
    from paper_2510_01119_amd.train import LR_POSITION
    assert LR_POSITION == 1e-5 and LR_DEFAULTS["mean_xyz"][0] == 1e-5
    assert PRESETS["lite"]["lambda_static"] == 4.0 and PRESETS["lite"]["lambda_dynamic"] == 4.0
    assert PRESETS["full"]["lambda_static"] == 1.0 and PRESETS["full"]["lambda_dynamic"] is None
    for p in PRESETS.values():
        assert p["motion"] == "otsu" and p["voxel"] == "adaptive"


def test_sch_rates_and_groups():
    """The SCH colour's Adam groups: the constant coefficient at the RGB rate
    in colour units (the basis value Y_00 scales a coefficient's colour), the
    higher ones 20 times slower."""
    import math
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    assert np.isclose(LR_DEFAULTS["sch_dc"][0] * y00, LR_DEFAULTS["rgb"][0])
    assert np.isclose(LR_DEFAULTS["sch_rest"][0] * 20.0, LR_DEFAULTS["sch_dc"][0])
    cfg = adam_config(100, rows=["sch_dc"])
    assert cfg.rows == 1 and np.isclose(cfg.lr0[0], LR_DEFAULTS["sch_dc"][0])
