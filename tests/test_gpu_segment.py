"""gs4d_otsu_mask against the Otsu oracle, bit for bit: the chosen split
(threshold = k* / 256) and the mask, on bimodal maps of display size and
ragged sizes, a map with NaNs, a constant map (no split) and one value."""
import numpy as np
import pytest
import torch

from oracle import otsu as O
from paper_2510_01119_amd import gs4d as G

from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def _maps():
    rng = np.random.default_rng(5)
    a = np.clip(np.where(rng.uniform(0, 1, 518400) < 0.2, rng.normal(0.8, 0.1, 518400),
                         rng.normal(0.15, 0.1, 518400)), 0, 1)
    b = rng.uniform(0, 1, 1001)
    c = rng.beta(0.5, 0.5, 65537)
    c[::97] = np.nan
    return {"bimodal_960x540": a, "uniform_1001": b, "beta_nan_65537": c,
            "constant": np.full(4096, 0.3), "single": np.array([0.7])}


@pytest.mark.parametrize("name", list(_maps()))
def test_otsu_matches_oracle(name):
    need_gpu()
    x = _maps()[name].astype(np.float32)
    k_ref, m_ref = O.otsu(x)
    X = torch.from_numpy(x).cuda()
    thr = torch.zeros(1, device="cuda")
    mask = torch.zeros(x.size, dtype=torch.uint8, device="cuda")
    ws = torch.zeros(G.gs4d_otsu_workspace_size(), dtype=torch.uint8, device="cuda")
    for _ in range(2):   # a second call on the same workspace gives the same result
        G.gs4d_otsu_mask(X, thr, mask, ws)
        torch.cuda.synchronize()
        assert float(thr.item()) == np.float32(k_ref) / np.float32(256)
        assert np.array_equal(mask.cpu().numpy(), m_ref)


def test_pooled_threshold_applied_per_map():
    """One Otsu threshold over several maps pooled (gs4d_otsu_mask on their
    concatenation), applied to each map and to a map outside the pool by
    gs4d_threshold_mask: the oracle's bins against the oracle's k*, bit for
    bit (a NaN reads as 0; k* = 256, no split, masks nothing)."""
    need_gpu()
    rng = np.random.default_rng(9)
    maps = [np.clip(rng.normal(0.2 + 0.5 * (i % 2), 0.15, 20000), 0, 1).astype(np.float32)
            for i in range(5)]
    maps[3][::13] = np.nan
    pooled = np.concatenate(maps)
    k_ref, _ = O.otsu(pooled)
    thr = torch.zeros(1, device="cuda")
    ws = torch.zeros(G.gs4d_otsu_workspace_size(), dtype=torch.uint8, device="cuda")
    G.gs4d_otsu_mask(torch.from_numpy(pooled).cuda(), thr, None, ws)
    other = rng.uniform(0, 1, 777).astype(np.float32)
    for m in maps + [other]:
        mask = torch.full((m.size,), 9, dtype=torch.uint8, device="cuda")
        G.gs4d_threshold_mask(torch.from_numpy(m).cuda(), thr, mask)
        torch.cuda.synchronize()
        assert np.array_equal(mask.cpu().numpy(), (O.bins_of(m) >= k_ref).astype(np.uint8))
    # no split: k* = 256, nothing is dynamic
    const = np.full(1000, 0.4, np.float32)
    G.gs4d_otsu_mask(torch.from_numpy(const).cuda(), thr, None, ws)
    mask = torch.full((other.size,), 9, dtype=torch.uint8, device="cuda")
    G.gs4d_threshold_mask(torch.from_numpy(other).cuda(), thr, mask)
    torch.cuda.synchronize()
    assert float(thr.item()) == 1.0 and int(mask.sum().item()) == 0
