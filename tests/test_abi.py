"""The C-ABI library loads and exports every entry point that include/gs4d.h
declares; host-side argument validation rejects bad calls without launching
anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gs4d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(gs4d_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2510_01119_amd import gs4d
    if not os.path.exists(gs4d.LIB_PATH):
        pytest.fail("libgs4d.so is not built (run paper_2510_01119_amd/build.py)")
    return gs4d.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2510_01119_amd import gs4d
    assert set(gs4d.EXPORTED) == set(_declared())


def test_status_strings(lib):
    assert lib.gs4d_status_string(0) == b"ok"
    assert lib.gs4d_status_string(-1) == b"invalid argument"
    assert lib.gs4d_version() >= 1


def test_invalid_arguments_rejected_on_host(lib):
    from paper_2510_01119_amd import gs4d, synth
    views = gs4d.make_views(synth.front_view(64, 64))
    # n_views out of range
    st = lib.gs4d_preprocess(None, 10, views, 0, None, None, None, None)
    assert st == -1 and b"n_views" in lib.gs4d_last_error()
    st = lib.gs4d_preprocess(None, 10, views, 17, None, None, None, None)
    assert st == -1
    # null pointers with n > 0
    st = lib.gs4d_preprocess(None, 10, views, 1, None, None, None, None)
    assert st == -1 and b"null" in lib.gs4d_last_error()
    # negative n
    st = lib.gs4d_preprocess(None, -1, views, 1, None, None, None, None)
    assert st == -1
    # views of different sizes
    two = gs4d.make_views(__import__("numpy").stack([synth.front_view(64, 64), synth.front_view(32, 32)]))
    st = lib.gs4d_preprocess(None, 0, two, 2, None, None, None, None)
    assert st == -1 and b"width" in lib.gs4d_last_error()
    # non-positive focal length
    bad = gs4d.make_views(synth.front_view(64, 64))
    bad[0].fx = 0.0
    assert lib.gs4d_preprocess(None, 0, bad, 1, None, None, None, None) == -1
    # bin_sort: workspace too small
    d = ctypes.c_void_p(1)
    st = lib.gs4d_bin_sort(d, d, d, 10, views, 1, 100, d, d, d, d, d, d, 16, None)
    assert st == -1 and b"workspace" in lib.gs4d_last_error()
    # render: unsupported batch
    opts = gs4d.gs4d_render_opts()
    opts.batch = 100
    st = lib.gs4d_render_fwd(d, 10, d, d, views, 1, ctypes.byref(opts), d, d, d, None)
    assert st == -1 and b"batch" in lib.gs4d_last_error()
    # prune: bad k_attr / min_count
    st = lib.gs4d_grid_prune(d, d, 99, None, 10, 0.1, 0.1, 1, 10, d, d, d, d, d, d, d, 1 << 30, None)
    assert st == -1
    st = lib.gs4d_grid_prune(d, None, 0, None, 10, 0.1, 0.1, 0, 10, d, d, d, d, d, d, d, 1 << 30, None)
    assert st == -1
    # adam: rows out of range
    cfg = gs4d.gs4d_adam_cfg()
    cfg.rows = 21
    assert lib.gs4d_adam_step(d, d, d, d, 10, ctypes.byref(cfg), d, None) == -1
    # ssim: bad shape
    assert lib.gs4d_ssim(d, d, 0, 3, 8, 8, 1.0, d, None, None, 0, None) == -1
    # SCH: degree, frequencies, period, reserved word; row counts
    assert lib.gs4d_sch_rows(3, 2) == 3 * 3 * 16
    assert lib.gs4d_sch_rows(0, 0) == 3
    assert lib.gs4d_sch_rows(4, 0) == -1 and lib.gs4d_sch_rows(0, 3) == -1
    for deg, nf, per, res in ((4, 0, 1.0, 0), (0, -1, 1.0, 0), (1, 1, 0.0, 0),
                              (1, 1, float("inf"), 0), (1, 1, 1.0, 7)):
        sch = gs4d.gs4d_sch()
        sch.degree, sch.n_freq, sch.period, sch.reserved = deg, nf, per, res
        st = lib.gs4d_preprocess_sch(d, d, 10, ctypes.byref(sch), views, 1, d, d, d, None)
        assert st == -1 and b"SCH" in lib.gs4d_last_error() or b"reserved" in lib.gs4d_last_error()
        st = lib.gs4d_preprocess_sch_bwd(d, d, 10, ctypes.byref(sch), views, 1, d, d, d, d, None)
        assert st == -1
    sch = gs4d.make_sch(2, 1, 2.0)
    st = lib.gs4d_preprocess_sch_bwd(d, d, 10, ctypes.byref(sch), views, 1, d, d, d, None, None)
    assert st == -1 and b"null" in lib.gs4d_last_error()
    assert lib.gs4d_sch_from_rgb(d, 5, 10, ctypes.byref(sch), d, None) == -1
    # binning strategies 0-3 (auto, per-tile radix, presort, counting)
    for strategy in (gs4d.BIN_COUNT, gs4d.BIN_PRESORT, gs4d.BIN_PER_TILE, gs4d.BIN_AUTO):
        assert lib.gs4d_set_bin_strategy(strategy) == 0
    assert lib.gs4d_set_bin_strategy(4) == -1 and b"strategy" in lib.gs4d_last_error()
    assert lib.gs4d_set_bin_strategy(-1) == -1
    assert lib.gs4d_set_bin_strategy(gs4d.BIN_AUTO) == 0


def test_workspace_queries(lib):
    a = lib.gs4d_bin_sort_workspace_size(1000, 1, 10000)
    b = lib.gs4d_bin_sort_workspace_size(1000, 1, 100000)
    assert b > a > 0
    # room for the counting strategy's per-tile counts: 8 columns of 4 B plus
    # a row total for each of up to 8,192 tiles per view
    for views in (1, 3):
        assert lib.gs4d_bin_sort_workspace_size(10, views, 0) >= views * 8192 * 36
    assert lib.gs4d_render_bwd_workspace_size(1000, 2) >= 1000 * 2 * 9 * 4
    assert lib.gs4d_grid_prune_workspace_size(10 ** 6, 5) > 10 ** 6 * 24
    assert lib.gs4d_ssim_workspace_size(1, 3, 64, 64) >= 3 * 3 * 64 * 64 * 4


def test_workspace_sizes_monotone(lib):
    """Workspace sizes never shrink as the capacity grows, also across the
    sizes where the radix sort and the scans switch to longer blocks (a
    smaller input may use shorter blocks, hence more block counts)."""
    caps = sorted({c + d for c in (1 << 10, 1 << 18, 1 << 20, 1 << 22, 1 << 24)
                   for d in (-1, 0, 1)})
    prev = 0
    for cap in caps:
        ws = lib.gs4d_bin_sort_workspace_size(1 << 17, 1, cap)
        assert ws >= prev, cap
        # the sort keeps one 256-count histogram per block of at most
        # 4,096 keys, at least
        assert ws >= cap * 12 + (cap // 4096) * 256 * 4, cap
        prev = ws
    for f in (lambda m: lib.gs4d_grid_prune_workspace_size(m, 3), lib.gs4d_knn8_workspace_size):
        prev = 0
        for m in caps:
            ws = f(m)
            assert ws >= prev, m
            prev = ws
