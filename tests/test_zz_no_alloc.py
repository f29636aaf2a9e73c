"""The allocation-free outer-volume entry point against obbv_outer_volume,
through the C ABI (needs an MI355X).  Two calls in a row, the second with a
smaller input: the fixed scratch array keeps the first call's contents, which
the second must not see."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def test_noalloc_equals_pooled_call_twice_second_smaller(api):
    import torch
    V, F = synth.noisy_torus(nu=128, nv=64)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    c, a, h = synth.random_boxes(48, seed=91, center_range=1.1, half_range=(0.1, 0.8))
    h[5] = np.nan                     # a non-finite box: NaN and a status bit
    B = torch.from_numpy(synth.boxes_to_array(c, a, h)).cuda()
    key = torch.from_numpy((np.arange(48) * 3 + 1).astype(np.int32)).cuda()
    for n, R in ((48, 96), (17, 40)):
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        got = api.outer_volume_noalloc(Vt, Ft, B[:n].contiguous(), R, seed=4, box_key=key[:n].contiguous(),
                                       status=status)
        ref = api.outer_volume(Vt, Ft, B[:n].contiguous(), R, seed=4, box_key=key[:n].contiguous())
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isnan(g[5]) and np.isnan(r[5])
        ok = ~np.isnan(r)
        assert np.array_equal(g[ok], r[ok]), (n, R)
        assert int(status.item()) & 0x1
    api.status()  # clear the pooled call's status bit


def test_noalloc_large_call_is_rejected_without_running(api):
    import torch
    V, F = synth.noisy_torus()
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    B = torch.zeros((200_000, 15), dtype=torch.float32, device="cuda")
    with pytest.raises(api.ObbvError) as e:
        api.outer_volume_noalloc(Vt, Ft, B, 32)
    assert e.value.code == -5
