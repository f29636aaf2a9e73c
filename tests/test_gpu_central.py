"""The central-projection estimator on the device (obbv_outer_volume_central)
against the central-projection oracle (Sec. 4.1, Eq. 9-10), through the C ABI
(needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import central, exact

from conftest import record_parity

pytestmark = pytest.mark.gpu

# Both sides take every crossing decision and depth in float64 with one order of
# operations; only the order of the final sum over the cones differs.
TOL_REL = 1e-11


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("m", [3, 8, 16, 32])
def test_central_estimator_matches_the_oracle(api, m):
    """Random boxes over the icosphere plus a box inside the solid (exactly 0),
    one far away and one holding the whole mesh, across more than one tile of
    triangles and a ragged last ray chunk: |gpu - oracle| <= 1e-11 (V_box + 1).
    With m = 3 and 8 every ray block spans two cube faces (no culling); with
    m = 16 a block is one face and with m = 32 a quarter of one, where the
    triangles outside the block's pyramid of directions are skipped."""
    V, F = synth.icosphere(3)
    c, a, h = synth.random_boxes(10, seed=23, center_range=0.8, half_range=(0.1, 0.7))
    c = np.concatenate([c, [[0.05, 0.0, -0.02], [4.0, 0.0, 0.0], [0.0, 0.0, 0.0]]]).astype(np.float32)
    a = np.concatenate([a, np.repeat(np.eye(3, dtype=np.float32)[None], 3, axis=0)]).astype(np.float32)
    h = np.concatenate([h, [[0.2, 0.2, 0.2], [0.3, 0.2, 0.4], [1.2, 1.1, 1.3]]]).astype(np.float32)
    B = _t(synth.boxes_to_array(c, a, h))
    api.status()
    got = api.outer_volume_central(_t(V), _t(F), B, m).cpu().numpy()
    assert api.status() == 0
    worst = 0.0
    for i in range(len(c)):
        want = central.obv(V, F, c[i], a[i], h[i], m)
        vb = exact.box_volume(h[i])
        err = abs(got[i] - want)
        worst = max(worst, err / (vb + 1.0))
        assert err <= TOL_REL * (vb + 1.0), (m, i, got[i], want)
    assert got[10] == 0.0
    record_parity({"test": f"central_estimator_m{m}", "boxes": len(c), "max_err_rel": worst})


def test_central_estimator_converges_and_flags(api):
    """On the torus the estimate approaches the exact outer volume as m grows
    (mean error relative to V_box falls from m = 8 to m = 32 and is below 2e-3
    at 32); NaN boxes give NaN with the NaN-box bit; repeated calls give the
    same bits."""
    V, F = synth.noisy_torus(nu=64, nv=32)
    c, a, h = synth.random_boxes(8, seed=29, center_range=1.0, half_range=(0.2, 0.6))
    h[5] = [0.3, -0.2, 0.3]
    B = _t(synth.boxes_to_array(c, a, h))
    Vt, Ft = _t(V), _t(F)
    ex = api.outer_volume_exact(Vt, Ft, B, axis=0).cpu().numpy()
    vb = 8.0 * h[:, 0].astype(np.float64) * h[:, 1] * h[:, 2]
    ok = np.arange(8) != 5
    api.status()
    err = {}
    for m in (8, 32):
        est = api.outer_volume_central(Vt, Ft, B, m).cpu().numpy()
        assert np.isnan(est[5])
        err[m] = float(np.mean(np.abs(est[ok] - ex[ok]) / vb[ok]))
    assert api.status() & 0x1
    assert err[32] < err[8] and err[32] < 2e-3
    again = api.outer_volume_central(Vt, Ft, B, 32).cpu().numpy()
    assert np.array_equal(again, est, equal_nan=True)


def test_central_estimator_edge_cases(api):
    """No boxes: nothing to do, no error.  A mesh without triangles: every cone
    lies outside, and the estimate is the cones' total volume (the oracle's, a
    little above V_box).  A flat box: exactly 0.  A triangle whose index is past
    the vertex count is skipped and sets OBBV_STATUS_BAD_INDEX: the estimate is
    the oracle's without that triangle."""
    V, F = synth.icosphere(2)
    c = np.array([[0.1, 0.0, 0.05], [0.1, 0.0, 0.05], [-0.3, 0.2, 0.1]], np.float32)
    a = np.repeat(np.eye(3, dtype=np.float32)[None], 3, axis=0)
    h = np.array([[0.5, 0.4, 0.3], [0.5, 0.0, 0.3], [0.6, 0.5, 0.7]], np.float32)
    B = _t(synth.boxes_to_array(c, a, h))
    m = 4
    api.status()
    none = api.outer_volume_central(_t(V), _t(F), B[:0], m)
    assert none.shape == (0,) and api.status() == 0
    empty = api.outer_volume_central(_t(V), _t(F[:0]), B, m).cpu().numpy()
    assert api.status() == 0
    for i in (0, 2):
        want = central.obv(V, F[:0], c[i], a[i], h[i], m)
        assert abs(empty[i] - want) <= TOL_REL * (exact.box_volume(h[i]) + 1.0), (i, empty[i], want)
    assert empty[1] == 0.0
    Fb = F.copy()
    Fb[7, 1] = len(V) + 5
    got = api.outer_volume_central(_t(V), _t(Fb), B, m).cpu().numpy()
    assert api.status() & 0x2
    keep = np.ones(len(F), bool)
    keep[7] = False
    for i in (0, 2):
        want = central.obv(V, F[keep], c[i], a[i], h[i], m)
        assert abs(got[i] - want) <= TOL_REL * (exact.box_volume(h[i]) + 1.0), (i, got[i], want)
    assert got[1] == 0.0


@pytest.mark.parametrize("m", [16, 24, 32])
def test_central_culling_gives_the_same_bits(api, monkeypatch, m):
    """Skipping the triangles that lie outside a ray block's pyramid of
    directions (OBBV_CENTRAL_CULL, on by default) changes no bit of the
    estimate: 65,536 triangles of the noisy torus, boxes of several sizes
    around it (m = 24 mixes blocks inside one face and blocks spanning two)."""
    V, F = synth.noisy_torus()
    c, a, h = synth.random_boxes(12, seed=31, center_range=1.1, half_range=(0.05, 0.8))
    B = _t(synth.boxes_to_array(c, a, h))
    Vt, Ft = _t(V), _t(F)
    api.status()  # clear what earlier calls left
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("OBBV_CENTRAL_CULL", flag)
        out[flag] = api.outer_volume_central(Vt, Ft, B, m).cpu().numpy()
    assert api.status() == 0
    assert np.array_equal(out["1"].view(np.int64), out["0"].view(np.int64)), m
    assert np.all(np.isfinite(out["1"]))
