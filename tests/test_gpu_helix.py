"""Large single mesh at full size: the capped helix tube (2,000,384 triangles),
a 7-level tree of covariance boxes (1 + 4 + ... + 4^6 = 5,461 nodes, 4,096 leaves)
and rays shrinking from 256 x 256 at the root to 32 x 32 at the leaves.
Needs an MI355X."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import raygrid

pytestmark = pytest.mark.gpu

LEVELS, BRANCH, SEED = 7, 4, 43
TOL_BOX = 1e-5


def level_R(level, R0=256):
    """256 * 2^(-level/2) rounded to a multiple of 8: 256, 184, 128, 88, 64, 48, 32."""
    return int(8 * round(R0 * 2.0 ** (-level / 2.0) / 8.0))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tree():
    """Top-down tree: every node's triangles are cut into `BRANCH` equal-count
    slices along the longest axis of the node's covariance box (centroid order)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2203_10521_amd import api
    t0 = time.perf_counter()
    V, F = synth.helix_tube()
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    cen = V.astype(np.float64)[F].mean(axis=1)
    nt = F.shape[0]
    cluster = np.zeros(nt, np.int64)
    levels = []
    for lv in range(LEVELS):
        n = BRANCH ** lv
        boxes, _ = api.fit(Vt, Ft, torch.from_numpy(cluster.astype(np.int32)).cuda(), n)
        B = boxes.cpu().numpy()
        levels.append((B, cluster.copy()))
        if lv + 1 == LEVELS:
            break
        # split each node along its longest axis into BRANCH equal-count parts
        longest = np.argmax(B[:, 12:15], axis=1)
        axis = B[:, 3:12].reshape(-1, 3, 3)[np.arange(n), longest]          # [n, 3]
        proj = np.einsum("ij,ij->i", cen, axis[cluster])
        order = np.lexsort((np.arange(nt), proj, cluster))
        counts = np.bincount(cluster, minlength=n)
        start = np.concatenate([[0], np.cumsum(counts)[:-1]])
        rank = np.empty(nt, np.int64)
        rank[order] = np.arange(nt) - np.repeat(start, counts)
        part = np.minimum(rank * BRANCH // np.maximum(counts[cluster], 1), BRANCH - 1)
        cluster = cluster * BRANCH + part
    _say(f"helix tree: {nt} triangles, {sum(len(b) for b, _ in levels)} nodes, "
         f"built in {time.perf_counter() - t0:.1f} s")
    return api, V, F, Vt, Ft, levels


def test_helix_tree_levels_evaluate_and_match_oracle_samples(tree):
    import torch
    api, V, F, Vt, Ft, levels = tree
    node0 = 0
    checked = []
    for lv, (B, cluster) in enumerate(levels):
        R = level_R(lv)
        n = len(B)
        Bt = torch.from_numpy(B).cuda()
        key = torch.arange(node0, node0 + n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obv = api.outer_volume(Vt, Ft, Bt, R, seed=SEED, box_key=key)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert api.status() == 0
        obv = obv.cpu().numpy()
        vb = 8.0 * B[:, 12].astype(np.float64) * B[:, 13] * B[:, 14]
        assert np.all(obv >= 0.0) and np.all(obv <= vb * (1 + 1e-12))
        # a covariance box encloses its cluster: the inside part is never empty
        assert np.all(obv < vb)
        _say(f"level {lv}: {n} boxes, R = {R}, {dt * 1e3:.1f} ms, "
             f"sum OBV {obv.sum():.5f}, sum V_box {vb.sum():.5f}")
        for j in sorted({n // 3, n - 1}):
            checked.append((lv, j, node0 + j, R, B[j], obv[j]))
        node0 += n
    worst = 0.0
    for lv, j, key, R, bx, got in checked:
        t0 = time.perf_counter()
        ref = raygrid.raygrid_obv(V, F, bx[:3], bx[3:12].reshape(3, 3), bx[12:15], R, SEED, key)
        err = abs(got - ref["obv"]) / ref["v_box"]
        worst = max(worst, err)
        _say(f"  oracle level {lv} node {j}: rel err {err:.2e} ({time.perf_counter() - t0:.1f} s)")
        assert err <= TOL_BOX, (lv, j, got, ref["obv"])
    _say(f"helix sampled boxes: worst |gpu - oracle| / V_box = {worst:.2e}")


def test_level_R_schedule():
    assert [level_R(lv) for lv in range(7)] == [256, 184, 128, 88, 64, 48, 32]
