"""kt_profile_enable / kt_profile_read: per-class launch timing with a class mask."""
import pytest

from paper_1608_06577_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kt():
    import torch
    assert torch.cuda.is_available()
    from paper_1608_06577_amd import kt as K
    K.lib()
    return K


def test_profile_class_mask(kt):
    w = I.workload_hotspot(nx=40, ny=36, neta=12, dx=0.5, deta=0.6, n_hot=30, seed=4)
    s = kt.Solver(w.grid, w.config, w.eos, w.prims)
    # every class: two launches of each per step
    s.profile(True)
    s.step(3)
    p = s.profile_read()
    for c in kt.PROFILE_CLASSES:
        assert p[c + "_launches"] == 6, (c, p)
        assert p[c + "_ms"] > 0.0
    # one class only
    s.profile(True, classes=("faces",))
    s.step(2)
    p = s.profile_read()
    assert p["faces_launches"] == 4 and p["faces_ms"] > 0.0
    assert all(p[c + "_launches"] == 0 for c in kt.PROFILE_CLASSES if c != "faces"), p
    # off: nothing recorded; reading resets
    s.profile(False)
    s.step(1)
    p = s.profile_read()
    assert all(p[c + "_launches"] == 0 for c in kt.PROFILE_CLASSES), p
    # masks outside 0..15 are rejected
    with pytest.raises(kt.KtError) as ei:
        kt._check(kt.lib().kt_profile_enable(s.ctx, 16), s.ctx)
    assert ei.value.status == kt.KT_E_ARG
    s.close()
