"""Planned (autotuned, graph-replayed) evaluations vs the eager call (needs an MI355X)."""
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


def _batch(n_meshes=6, boxes_per_mesh=64, seed=0):
    import torch
    g = np.random.default_rng(seed)
    meshes, boxes, bm = [], [], []
    for m in range(n_meshes):
        n = int(g.integers(12, 30))
        V, F = synth.noisy_cube_sphere(n, seed=300 + m)
        meshes.append((torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()))
        c, a, h = synth.random_boxes(boxes_per_mesh, seed=400 + m, center_range=1.0, half_range=(0.1, 0.6))
        boxes.append(synth.boxes_to_array(c, a, h))
        bm += [m] * boxes_per_mesh
    B = torch.from_numpy(np.concatenate(boxes)).cuda()
    return meshes, B, torch.from_numpy(np.array(bm, np.int32)).cuda()


def test_plan_replays_equal_eager_calls(api):
    import torch
    meshes, B, bm = _batch()
    plan = api.OuterVolumePlan(B, 32, seed=3, meshes=meshes, box_mesh=bm, headroom=1.5)
    info = plan.info()
    assert info["block_rays"] in (2048, 4096, 8192) and min(info["tuned_ms"]) > 0
    eager = api.outer_volume_ex(None, None, B, 32, seed=3, block_rays=info["block_rays"], meshes=meshes,
                                box_mesh=bm)["obv"].cpu().numpy()
    api.status()
    for rep in range(4):
        got = plan.launch().clone()
        # eager work and a synchronisation between replays
        again = api.outer_volume_ex(None, None, B, 32, seed=3, block_rays=info["block_rays"], meshes=meshes,
                                    box_mesh=bm)["obv"]
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), eager), rep
        assert np.array_equal(again.cpu().numpy(), eager)
    assert api.status() == 0
    # new box contents, same arrays: the replay follows them
    B[:, :3] += 0.05
    got = plan.launch().cpu().numpy()
    ref = api.outer_volume_ex(None, None, B, 32, seed=3, block_rays=info["block_rays"], meshes=meshes,
                              box_mesh=bm)["obv"].cpu().numpy()
    assert api.status() == 0
    assert np.array_equal(got, ref)
    plan.close()


def test_plan_follows_grown_boxes(api):
    """The plan keeps no per-triangle records in device memory, so boxes grown
    after planning (three times larger) are still evaluated in full: the replay
    equals the eager call and raises no status bit."""
    import torch
    meshes, B, bm = _batch(n_meshes=2, boxes_per_mesh=32, seed=1)
    plan = api.OuterVolumePlan(B, 32, seed=3, meshes=meshes, box_mesh=bm, headroom=1.0, block_rays=2048)
    api.status()
    B[:, 12:] *= 3.0
    got = plan.launch().clone()
    torch.cuda.synchronize()
    assert api.status() == 0
    ref = api.outer_volume_ex(None, None, B, 32, seed=3, meshes=meshes, box_mesh=bm)["obv"]
    assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
    plan.close()
