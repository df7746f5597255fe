"""Tuning table: host logic only (no GPU needed)."""
import json

import pytest


def _msadp():
    from paper_2601_15458_amd import msadp
    return msadp


@pytest.fixture(autouse=True)
def _clean():
    M = _msadp()
    M.tune_clear()
    yield
    M.tune_clear()


def test_candidates():
    M = _msadp()
    assert M.tune_candidates(M.MSA_TUNE_LEV) == [4, 8, 16, 20, 24, 28, 32]
    assert M.tune_candidates(M.MSA_TUNE_NW) == [16, 32, 64]
    assert M.tune_candidates(M.MSA_TUNE_TREE) == [4, 8, 16, 20, 24, 32]
    assert M.tune_candidates(M.MSA_TUNE_PAIRS) == [1, 2, 64]
    xl = M.tune_candidates(M.MSA_TUNE_TREE_XL)
    assert M.xl_value(1, 0, 0) in xl and M.xl_value(2, 128, M.XL_CAP_ALL) in xl
    assert all(v >> 28 in (1, 2) for v in xl)


def test_set_get_clear():
    M = _msadp()
    assert M.tune_get(M.MSA_TUNE_LEV, 4, 25) == 0
    M.tune_set(M.MSA_TUNE_LEV, 4, 25, 28)
    M.tune_set(M.MSA_TUNE_NW, 4, 3, 64)
    M.tune_set(M.MSA_TUNE_TREE, 20, 32, 16)
    assert M.tune_get(M.MSA_TUNE_LEV, 4, 25) == 28
    assert M.tune_get(M.MSA_TUNE_TREE, 20, 32) == 16
    assert M.tune_get(M.MSA_TUNE_TREE, 4, 25) == 0
    assert M.tune_get(M.MSA_TUNE_LEV, 5, 25) == 0
    assert M.tune_get(M.MSA_TUNE_NW, 4, 3) == 64
    M.tune_clear()
    assert M.tune_get(M.MSA_TUNE_LEV, 4, 25) == 0


@pytest.mark.parametrize("kind,sigma,bin_,value", [
    (0, 4, 25, 30),      # not a word class
    (1, 4, 3, 48),       # not a barrier interval
    (2, 4, 3, 28),       # a pair-kernel class the tree build does not have
    (3, 4, 3, 32),       # not a pair layout (1, 2 or 64)
    (5, 4, 3, 1),        # unknown kind
    (4, 4, 3, 0),        # across-lanes value with no words per lane
    (4, 4, 3, 3 << 28),  # three words per lane (the tree passes have 1 or 2)
    (0, 1, 3, 32),       # alphabet too small
    (0, 4, 0, 32),       # empty bin
])
def test_invalid_entries(kind, sigma, bin_, value):
    M = _msadp()
    with pytest.raises(M.MsaError) as ex:
        M.tune_set(kind, sigma, bin_, value)
    assert ex.value.code == M.MSA_EINVAL


def test_export_import_round_trip():
    M = _msadp()
    M.tune_set(M.MSA_TUNE_LEV, 4, 25, 28)
    M.tune_set(M.MSA_TUNE_LEV, 20, 3, 4)
    M.tune_set(M.MSA_TUNE_NW, 4, 5, 16)
    M.tune_set(M.MSA_TUNE_TREE, 20, 32, 24)
    M.tune_set(M.MSA_TUNE_PAIRS, 4, 160, 2)
    xv = M.xl_value(2, 256, M.XL_CAP_ALL)
    M.tune_set(M.MSA_TUNE_TREE_XL, 4, 8, xv)
    text = M.tune_export()
    doc = json.loads(text)
    assert sorted(map(tuple, doc["entries"])) == [(0, 4, 25, 28), (0, 20, 3, 4), (1, 4, 5, 16),
                                                  (2, 20, 32, 24), (3, 4, 160, 2),
                                                  (4, 4, 8, xv)]
    M.tune_clear()
    M.tune_import(text)
    assert M.tune_get(M.MSA_TUNE_LEV, 4, 25) == 28
    assert M.tune_get(M.MSA_TUNE_LEV, 20, 3) == 4
    assert M.tune_get(M.MSA_TUNE_NW, 4, 5) == 16
    assert M.tune_get(M.MSA_TUNE_TREE, 20, 32) == 24
    assert M.tune_get(M.MSA_TUNE_PAIRS, 4, 160) == 2
    assert M.tune_get(M.MSA_TUNE_TREE_XL, 4, 8) == xv
    assert "sums up to 256, poles up to all" in M.xl_describe(xv)


def test_import_rejects_other_arch_and_bad_entries():
    M = _msadp()
    arch = json.loads(M.tune_export())["arch"]
    M.tune_set(M.MSA_TUNE_LEV, 4, 25, 28)
    bad = [json.dumps({"arch": arch + "x", "entries": [[0, 4, 25, 16]]}),
           json.dumps({"arch": arch, "entries": [[0, 4, 25, 17]]}),
           json.dumps({"arch": arch, "entries": [[0, 4, 25]]}),
           "not json"]
    for text in bad:
        with pytest.raises(M.MsaError) as ex:
            M.tune_import(text)
        assert ex.value.code == M.MSA_EINVAL
    assert M.tune_get(M.MSA_TUNE_LEV, 4, 25) == 28      # unchanged


def test_save_and_load(tmp_path):
    M = _msadp()
    M.tune_set(M.MSA_TUNE_NW, 4, 2, 64)
    path = str(tmp_path / "tune.json")
    M.tune_save(path)
    M.tune_clear()
    assert M.tune_load(path)
    assert M.tune_get(M.MSA_TUNE_NW, 4, 2) == 64
    assert not M.tune_load(str(tmp_path / "missing.json"))


def test_calibration_fit_offset():
    """The ranking offset of the pruned median is a host-side fit (its value
    is a parameter of tree_build_pruned): intercept over slope of the line
    through (predicted, true) distances, clipped; the length prior (cap)
    when the predictor carries no signal."""
    import numpy as np
    from paper_2601_15458_amd.learned import fit_offset
    yh = np.linspace(0.1, 2.0, 50)
    off, a, b, r = fit_offset(yh, 0.3 + 0.5 * yh)
    assert abs(a - 0.3) < 1e-12 and abs(b - 0.5) < 1e-12 and abs(off - 0.6) < 1e-12
    assert abs(r - 1.0) < 1e-12
    # noise around the same line keeps the offset near a / b
    rng = np.random.default_rng(3)
    off, _, _, r = fit_offset(yh, 0.3 + 0.5 * yh + rng.normal(0, 0.01, 50))
    assert abs(off - 0.6) < 0.05 and r > 0.99
    # negative slope, a constant predictor, a negative intercept, the cap
    assert fit_offset(yh, 1.0 - 0.2 * yh, cap=7.0)[0] == 7.0
    assert fit_offset(np.ones(10), np.arange(10.0), cap=5.0)[0] == 5.0
    assert fit_offset(yh, -1.0 + yh)[0] == 0.0
    assert fit_offset(yh, 100.0 + 0.01 * yh, cap=64.0)[0] == 64.0
