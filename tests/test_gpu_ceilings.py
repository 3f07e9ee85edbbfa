"""The ceiling measurement runs, loses no insert and returns plausible rates."""
import pytest

import paper_2505_04431_amd as kc

pytestmark = pytest.mark.gpu


def test_measure_ceilings():
    c = kc.kc.measure_ceilings(1 << 30)
    assert c["lost"] == 0
    assert 500 < c["copy_gbs"] < 9000
    assert 0.5 < c["hbm_insert_gops"] < c["lds_insert_gops"]
    assert c["mall_insert_gops"] > 0.5
    with pytest.raises(kc.KcError):
        kc.kc.measure_ceilings(1 << 20)
