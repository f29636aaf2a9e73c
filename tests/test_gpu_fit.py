"""HIP covariance OBB fit vs the CPU oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import synth
from oracle import fit as ofit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api as A
    return A


@pytest.mark.parametrize("nclusters", [1, 7, 64])
def test_fit_clusters_torus(api, nclusters):
    import torch
    V, F = synth.noisy_torus(nu=128, nv=64)
    # contiguous strips of the torus grid as clusters, one cluster id left empty, some triangles unassigned
    cl = (np.arange(len(F)) * nclusters // len(F)).astype(np.int32)
    cl[::97] = -1
    if nclusters > 2:
        cl[cl == 1] = 0
    boxes, eig = api.fit(torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda(), torch.from_numpy(cl).cuda(),
                         nclusters)
    boxes = boxes.cpu().numpy().astype(np.float64)
    eig = eig.cpu().numpy()
    ref = ofit.fit_clusters(V, F, cl, nclusters)
    for k in range(nclusters):
        c0, Q0, h0, l0 = ref[k]
        c1, Q1, h1 = boxes[k, :3], boxes[k, 3:12].reshape(3, 3), boxes[k, 12:]
        if not np.any(cl == k):
            assert np.all(h1 == 0) and np.allclose(Q1, np.eye(3))
            continue
        assert np.allclose(eig[k], l0, rtol=1e-9, atol=1e-15)
        vol0, vol1 = np.prod(h0), np.prod(h1)
        assert abs(vol1 - vol0) <= 1e-5 * vol0
        gaps = np.abs(np.diff(l0)) / max(l0[0], 1e-300)
        for i in range(3):
            well_separated = (i == 0 and gaps[0] > 1e-3) or (i == 2 and gaps[1] > 1e-3) or \
                             (i == 1 and gaps.min() > 1e-3)
            if well_separated:
                ang = np.arccos(min(1.0, abs(Q1[i] @ Q0[i]) / np.linalg.norm(Q1[i])))
                assert ang < 1e-4, (k, i, ang)
        assert np.allclose(c1, c0, atol=1e-5 * (1 + np.abs(c0).max()))
        # the fitted box encloses the cluster's vertices (float32 box, float64 check)
        idx = np.unique(F[cl == k])
        loc = (V[idx].astype(np.float64) - c1) @ Q1.T
        assert np.all(np.abs(loc) <= h1 * (1 + 1e-5) + 1e-6)


def test_fit_rotated_cuboid_exact_axes(api):
    import torch
    _, a, _ = synth.random_boxes(1, seed=5)
    half = np.array([0.9, 0.5, 0.2])
    V, F = synth.cuboid(half, (0.3, -0.2, 0.1), a[0])
    cl = np.zeros(len(F), np.int32)
    boxes, eig = api.fit(torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda(), torch.from_numpy(cl).cuda(), 1)
    b = boxes.cpu().numpy()[0].astype(np.float64)
    Q = b[3:12].reshape(3, 3)
    for i in range(3):
        assert abs(abs(Q[i] @ a[0][i].astype(np.float64)) - 1) < 1e-6
    assert np.allclose(b[12:], half, rtol=1e-5)


def test_fit_is_bitwise_independent_of_triangle_order(api):
    """Exact integer sums: the same clusters give bit-identical boxes and
    eigenvalues on a repeat, and with the triangles listed in another order
    (37 clusters interleaved at random, so every wave adds into several)."""
    import torch
    V, F = synth.noisy_torus(nu=128, nv=64)
    g = np.random.default_rng(3)
    cl = g.integers(-1, 37, size=len(F)).astype(np.int32)
    Vt = torch.from_numpy(V).cuda()

    def run(order):
        b, e = api.fit(Vt, torch.from_numpy(F[order]).cuda(), torch.from_numpy(cl[order]).cuda(), 37)
        return b.cpu().numpy(), e.cpu().numpy()

    ident = np.arange(len(F))
    b0, e0 = run(ident)
    for order in (ident, g.permutation(len(F)), ident[::-1].copy()):
        b1, e1 = run(order)
        assert np.array_equal(b0.view(np.uint32), b1.view(np.uint32))
        assert np.array_equal(e0.view(np.uint64), e1.view(np.uint64))
