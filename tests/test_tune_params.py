"""Launch parameters of the library (host only, no GPU): names, candidate
values, rejection of others, describe / save / load round trip."""
import os

import pytest

from paper_2306_09189_amd import hecnn

NAMES = {"ntt16_radix": [16, 2], "ntt_fp64": [1, 0], "ntt_row_vals": [16, 8], "ntt_tile": [2048, 4096, 8192], "ntt_group": [0, 64, 256, 1024],
         "ks_rot_batch": [4, 8, 16, 32], "ks_overlap": [0, 1], "ks_amounts": [1, 2, 4, 8, 16]}

pytestmark = pytest.mark.skipif(not os.path.exists(hecnn.LIB_PATH), reason="library not built")


@pytest.fixture
def restore():
    saved = {k: hecnn.tune_get(k) for k in NAMES}
    yield
    for k, v in saved.items():
        hecnn.tune_set(k, v)


def test_defaults_and_candidates(restore):
    assert {k: hecnn.tune_get(k) for k in NAMES} == {"ntt16_radix": 16, "ntt_fp64": 1, "ntt_row_vals": 16,
                                                       "ntt_tile": 4096, "ntt_group": 0,
                                                       "ks_rot_batch": 32, "ks_overlap": 0, "ks_amounts": 4}
    for k, vals in NAMES.items():
        for v in vals:
            hecnn.tune_set(k, v)
            assert hecnn.tune_get(k) == v
    with pytest.raises(hecnn.HecError):
        hecnn.tune_set("ntt_tile", 3000)
    with pytest.raises(hecnn.HecError):
        hecnn.tune_set("no_such_parameter", 1)


def test_save_load_roundtrip(restore, tmp_path):
    hecnn.tune_set("ntt16_radix", 2)
    hecnn.tune_set("ks_amounts", 8)
    p = tmp_path / "tune.txt"
    hecnn.tune_save(p)
    desc = hecnn.tune_describe()
    assert "ntt16_radix=2" in desc and "ks_amounts=8" in desc
    hecnn.tune_set("ntt16_radix", 16)
    hecnn.tune_set("ks_amounts", 1)
    hecnn.tune_load(p)
    assert hecnn.tune_get("ntt16_radix") == 2 and hecnn.tune_get("ks_amounts") == 8
    assert hecnn.tune_describe() == desc
