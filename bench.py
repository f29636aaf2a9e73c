"""Throughput of the outer-volume hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-legs] ...

Headline workload (the hierarchy configuration the metric is quoted on): the
noisy torus (R = 1, r = 0.35, 256 x 128 quads = 65,536 triangles, radial
displacement 0.02 x a smooth 8 x 8-mode Fourier field, seed 21); a 4-layer
hierarchy with branching 4 (1 / 4 / 16 / 64 boxes), 20 Lloyd iterations per
layer, 2 multigrid-like up / down sweeps, 128 x 128 rays per box face, K = 32
flood pops per group per round.  One step = one complete obbv_build_hierarchy.
`value` is box outer-volume evaluations per second over the build.

Other objects of the line:
  roofline      the cast kernel (cull, LDS rays, FP32 ray-triangle tests): 16
                FLOP per test the kernel performs, over the time during which a
                cast launch runs (HIP events around every launch, on the stream
                it is launched on; the floods of independent groups run on two
                streams whose launches overlap, so the launch intervals are
                merged), against the FP32 vector peak; the per-launch average
                beside it; `traffic` = its HBM bytes per launch from rocprofv3
                counters
  culling_stream  the bytes the cast kernel streams per launch (48 B per
                triangle-list entry per unit) as a rate against HBM, next to the
                algorithmic bytes of the calls (36 B per triangle + 68 B per box)
  legs          the other workloads: 64 boxes on the icosphere (R = 32), 256
                noisy spheres x 64 boxes in one planned launch (R = 64), the 2 M
                triangle helix's 5,461-node covariance tree (R 256 -> 32)
  obb_tree      per-layer sum of OBV of the built hierarchy vs the top-down
                covariance tree (the paper's Fig. 6 comparison)
  exact_evaluator  the exact clipped-prism evaluator on the hierarchy's boxes:
                calls per second and the deviation from it of the hot path's
                estimator and of the paper's central-projection estimator
  collision_queries  synthetic sphere queries against the built hierarchy and
                the covariance tree: sphere-box tests per query (the paper's
                collision experiment counts such tests)
  surrogate     the ranker trained on 1.05 M exact outer fractions of the batched
                workload's spheres 0-223, validated on 224-255 against the
                occupancy estimate (MAE, top-1 of flood-candidate groups); then
                the same hierarchy, and 2 Lloyd iterations on 16 held-out
                spheres, with network-ranked floods, occupancy-mean-ranked
                floods, and network-ranked floods verifying the top 4 per box
  cpu_baseline  the CPU oracle on a bounded sample of the hierarchy's boxes
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("box outer-volume evals/s + ray-tri tests/s (% FP32 peak); "
          "Lloyd moves/s surrogate vs exact")
FP32_PEAK_TFLOPS = 157.3            # MI355X FP32 vector, packed
FP32_NONPACKED_TFLOPS = 78.6        # the same without packed FP32 (this build's code)
HBM_PEAK_GBPS = 8000.0
FLOP_PER_TEST = 16                  # 3 edge functions x 2 FMA + depth plane 2 FMA
HIER = dict(levels=4, branching=4, iters=20, sweeps=2, R=128, seed=23, pops_per_round=32)
SEED_MESH = 21

# HBM traffic of the cast kernel per launch on this workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, then WRITE_SIZE, over the cast-kernel dispatches of one
# build), each scaled by the same counter's reading for a plain device copy of
# known size.  Valid only for the code it was measured on (the hash covers the
# outer-volume source and its shared header, comments and blank lines left
# out): any change to that code reports null until the counters are re-taken.
K_CAST_TRAFFIC = {"source_sha256": "25ff971cb1b98d1394db0913a2cdcb8a42e3b0ddd0966fbb1dc5f7f979e3d337",
                  "fetch_bytes_per_launch": 28134399, "write_bytes_per_launch": 35727,
                  "fetch_kib_raw": 13738.01, "write_kib_raw": 34.89,
                  "copy_factor_fetch": 1.99993, "copy_factor_write": 1.00000}
CAST_SOURCES = ("outer_volume.hip", "common.h")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cast_source_sha256():
    """sha256 of the cast kernel's sources with comments, blank lines and
    trailing spaces removed (the code the counters were taken on)."""
    import re
    h = hashlib.sha256()
    for name in CAST_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_10521_amd", "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def traffic_bytes():
    if K_CAST_TRAFFIC is None or cast_source_sha256() != K_CAST_TRAFFIC["source_sha256"]:
        return None
    return K_CAST_TRAFFIC["fetch_bytes_per_launch"] + K_CAST_TRAFFIC["write_bytes_per_launch"]


def kernel_rates(test_ms, launches, tests, nbytes):
    """Average cast launch (ms), tests per launch, FP32 rate (TFLOP/s) of the
    tests and the rate of the culling stream (GB/s)."""
    avg_ms = test_ms / max(launches, 1)
    per_launch = tests / max(launches, 1)
    tflops = per_launch * FLOP_PER_TEST / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    gbps = nbytes / max(launches, 1) / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return avg_ms, per_launch, tflops, gbps


def timed_profile(api, torch, fn, reps):
    """Runs fn reps times under the library's profile counters; returns
    (wall seconds, cast ms, launches, tests, bytes)."""
    fn()
    torch.cuda.synchronize()
    api.profile_enable(True)
    api.profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n, tests, nbytes = api.profile_read()
    api.profile_enable(False)
    return dt, ms, n, tests, nbytes


def leg_object(n_boxes, reps, dt, ms, n, tests, nbytes, **extra):
    avg_ms, per_launch, tflops, gbps = kernel_rates(ms, n, tests, nbytes)
    out = {"n_boxes": int(n_boxes), "evals_per_s": n_boxes * reps / dt, "ms_per_call": 1e3 * dt / reps,
           "cast_avg_ms": avg_ms, "tests_per_launch": per_launch,
           "tests_per_s": tests / (ms * 1e-3) if ms > 0 else None,
           "fp32_tflops": tflops, "fp32_frac": tflops / FP32_PEAK_TFLOPS,
           "culling_stream_gbps": gbps}
    out.update(extra)
    return out


def saturated(api, torch, Vt, Ft, boxes, R, seed):
    """One large evaluation: the hierarchy's boxes plus perturbed copies (4,096 boxes)."""
    g = np.random.default_rng(5)
    B = np.repeat(boxes, 4096 // len(boxes) + 1, axis=0)[:4096].copy()
    B[len(boxes):, :3] += g.normal(0, 0.05, size=(4096 - len(boxes), 3)).astype(np.float32)
    B[len(boxes):, 12:] *= g.uniform(0.8, 1.2, size=(4096 - len(boxes), 3)).astype(np.float32)
    Bt = torch.from_numpy(B).cuda()
    res = timed_profile(api, torch, lambda: api.outer_volume(Vt, Ft, Bt, R, seed=seed), 3)
    return leg_object(len(B), 3, *res, workload="the built hierarchy's boxes + perturbed copies, R=128")


def leg_config1(api, torch):
    import synth
    V, F = synth.icosphere(3)
    c, a, h = synth.random_boxes(64, seed=12)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    B = torch.from_numpy(synth.boxes_to_array(c, a, h)).cuda()
    res = timed_profile(api, torch, lambda: api.outer_volume(Vt, Ft, B, 32, seed=13), 50)
    return leg_object(64, 50, *res, workload="icosphere 1,280 triangles, 64 random boxes, R=32")


def exact_evaluator_leg(api, torch, Vt, Ft, boxes, R, seed):
    """The exact evaluator (clipped-prism integral, float64) on the built
    hierarchy's boxes against the torus, next to the estimator of the hot path
    on the same boxes: calls per second and the estimator's deviation."""
    B = torch.from_numpy(np.ascontiguousarray(boxes)).cuda()
    n = B.shape[0]
    api.outer_volume_exact(Vt, Ft, B, axis=0)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ex = api.outer_volume_exact(Vt, Ft, B, axis=0)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    est = api.outer_volume(Vt, Ft, B, R, seed=seed)
    torch.cuda.synchronize()
    e, x = est.cpu().numpy(), ex.cpu().numpy()
    h = boxes[:, 12:15].astype(np.float64)
    vb = 8.0 * h[:, 0] * h[:, 1] * h[:, 2]
    ok = vb > 0
    dev = np.abs(e - x)[ok] / vb[ok]
    # the paper's central-projection estimator on the same boxes (cube map 6 x 32 x 32)
    m = 32
    api.outer_volume_central(Vt, Ft, B[:1], m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cp = api.outer_volume_central(Vt, Ft, B, m)
    torch.cuda.synchronize()
    dtc = time.perf_counter() - t0
    cdev = np.abs(cp.cpu().numpy() - x)[ok] / vb[ok]
    return {"n_boxes": int(n), "ms_per_call": 1e3 * dt, "evals_per_s": n / dt,
            "pair_tests_per_s": n * int(Ft.shape[0]) / dt,
            "estimator_R": R, "estimator_dev_mean": float(dev.mean()), "estimator_dev_max": float(dev.max()),
            "central_m": m, "central_ms_per_call": 1e3 * dtc, "central_evals_per_s": n / dtc,
            "central_dev_mean": float(cdev.mean()), "central_dev_max": float(cdev.max()),
            "workload": "the built torus hierarchy's boxes, 65,536 triangles, cast axis 0, float64"}


def collision_leg(api, torch, V, Vt, Ft, out, hp, n_spheres=65536):
    """Synthetic collision queries (the stand-in for the paper's collision
    experiment): the same spheres against the built hierarchy and the top-down
    covariance tree; sphere-box tests per query and queries per second."""
    import synth
    L, b = hp["levels"], hp["branching"]
    tree = api.build_obb_tree(Vt, Ft, L, b)
    S = torch.from_numpy(synth.query_spheres(V, n_spheres, seed=77)).cuda()
    res = {}
    for name, boxes, tri_node in (("hierarchy", out["boxes"], out["tri_node"]),
                                  ("obb_tree", tree["boxes"], tree["tri_node"])):
        used = np.zeros(len(boxes), np.uint8)
        ids = tri_node[tri_node >= 0]
        used[ids] = 1
        B = torch.from_numpy(np.ascontiguousarray(boxes)).cuda()
        U = torch.from_numpy(used).cuda()
        api.collision_queries(B, L, b, S, node_used=U)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            tests, hits = api.collision_queries(B, L, b, S, node_used=U)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"tests_per_query": float(tests.double().mean()), "hits_per_query": float(hits.double().mean()),
                     "queries_per_s": n_spheres / dt}
    res["tests_ratio"] = res["hierarchy"]["tests_per_query"] / res["obb_tree"]["tests_per_query"]
    res["workload"] = (f"{n_spheres} spheres, centres uniform in the torus's bounding box grown by 20 %, radii "
                       "log-uniform in 1-20 % of its diagonal; 4 levels, branching 4")
    return res


def leg_config3(api, torch):
    import synth
    host = config3_meshes()
    gen_s = _CONFIG3["generation_s"]
    meshes, boxes, bm = [], [], []
    for m, (V, F) in enumerate(host):
        meshes.append((torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()))
        c, a, h = synth.random_boxes(64, seed=5000 + m)
        boxes.append(synth.boxes_to_array(c, a, h))
        bm += [m] * 64
    Bt = torch.from_numpy(np.concatenate(boxes)).cuda()
    bmt = torch.from_numpy(np.array(bm, np.int32)).cuda()
    plan = api.OuterVolumePlan(Bt, 64, seed=33, meshes=meshes, box_mesh=bmt)
    info = plan.info()
    # the plan is a graph: time its replays with events on the stream
    plan.launch()
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    plan.close()
    # the same call eager, under the profile counters (tests, cast time)
    res = timed_profile(api, torch, lambda: api.outer_volume_ex(None, None, Bt, 64, seed=33, meshes=meshes,
                                                                 box_mesh=bmt, block_rays=info["block_rays"]), 2)
    out = leg_object(len(Bt), 2, *res, workload="256 noisy spheres (8.35 M triangles), 64 boxes each, R=64")
    out.update({"planned_ms_per_launch": ms, "planned_evals_per_s": len(Bt) / (ms * 1e-3),
                "block_rays": info["block_rays"], "autotune_ms": info["tuned_ms"], "n_triangles":
                int(sum(F.shape[0] for _, F in host)), "generation_s": gen_s})
    return out


def leg_config4(api, torch):
    import synth
    V, F = synth.helix_tube()
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    t0 = time.perf_counter()
    tree = api.build_obb_tree(Vt, Ft, 7, 4)
    tree_s = time.perf_counter() - t0
    boxes = tree["boxes"]
    Rs = [256, 184, 128, 88, 64, 48, 32]
    total_ms = 0.0
    per_level = []
    base = 0
    api.profile_enable(True)
    api.profile_read()
    for lv, R in enumerate(Rs):
        n = 4 ** lv
        Bt = torch.from_numpy(boxes[base:base + n].copy()).cuda()
        key = torch.arange(base, base + n, dtype=torch.int32, device="cuda")
        api.outer_volume(Vt, Ft, Bt, R, seed=43, box_key=key)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        api.outer_volume(Vt, Ft, Bt, R, seed=43, box_key=key)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        total_ms += dt * 1e3
        per_level.append({"level": lv, "boxes": n, "R": R, "ms": dt * 1e3})
        base += n
    ms, launches, tests, nbytes = api.profile_read()
    api.profile_enable(False)
    avg_ms, per_launch, tflops, gbps = kernel_rates(ms, launches, tests, nbytes)
    return {"workload": "helix tube 2,000,384 triangles; 5,461-node covariance tree (obbv_build_obb_tree, 7 layers, "
                        "branching 4); R = 256, 184, 128, 88, 64, 48, 32 by layer",
            "n_boxes": int(len(boxes)), "evals_per_s": len(boxes) / (total_ms * 1e-3), "total_ms": total_ms,
            "tree_build_s": tree_s, "per_level": per_level, "tests_per_s": tests / (ms * 1e-3) if ms > 0 else None,
            "fp32_frac": tflops / FP32_PEAK_TFLOPS}


def obb_tree_comparison(api, torch, Vt, Ft, out, hp):
    """Per-layer sum of OBV: the built hierarchy vs the top-down covariance tree."""
    L, b = hp["levels"], hp["branching"]
    tree = api.build_obb_tree(Vt, Ft, L, b)
    key = torch.arange(len(tree["boxes"]), dtype=torch.int32, device="cuda")
    obv_t = api.outer_volume(Vt, Ft, torch.from_numpy(tree["boxes"]).cuda(), hp["R"], seed=hp["seed"],
                             box_key=key).cpu().numpy()
    hier, tr = [], []
    base = 0
    for lv in range(L):
        n = b ** lv
        used = np.array([(out["tri_node"][lv] == base + j).any() for j in range(n)])
        hier.append(float(out["obv"][base:base + n][used].sum()))
        tr.append(float(obv_t[base:base + n].sum()))
        base += n
    w = [L - lv for lv in range(L)]
    return {"per_layer_hierarchy": hier, "per_layer_obb_tree": tr,
            "e_hierarchy": float(sum(x * y for x, y in zip(w, hier))),
            "e_obb_tree": float(sum(x * y for x, y in zip(w, tr)))}


_CONFIG3 = {}


def config3_meshes():
    """The batched workload's 256 noisy spheres (generated once per run)."""
    import synth
    if "host" not in _CONFIG3:
        t0 = time.perf_counter()
        _CONFIG3["host"] = synth.noisy_sphere_batch(256, seed=3)
        _CONFIG3["generation_s"] = time.perf_counter() - t0
    return _CONFIG3["host"]


def ranker_eval_set(api, torch, V, F, seed, n_single, n_groups=64):
    """Random boxes around a mesh, then flood-candidate groups (a base box and 8
    copies grown by one more triangle each): inputs, exact fractions and OBVs."""
    import synth
    from paper_2203_10521_amd import ranker
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    base, cand = synth.flood_candidates(V, F, n_groups, seed=seed)
    B = torch.from_numpy(np.concatenate([synth.mixed_boxes(V, n_single, seed=seed + 1), base,
                                         cand.reshape(-1, 15)])).cuda()
    X, t, _ = ranker.make_dataset([(Vt, Ft)], [B], R=64, seed=1, nb=16)
    obv = api.outer_volume(Vt, Ft, B, 64, seed=1)
    return X, t, obv, B, n_single, len(base)


def lloyd_held_out(api, torch, host, ids, surrogates):
    """Two Lloyd iterations on each held-out mesh (8 k-means groups x 4 boxes,
    R = 64) per evaluation mode: moves per second and the summed layer error."""
    from paper_2203_10521_amd import ranker
    res = {name: {"moves": 0, "seconds": 0.0, "layer_error": 0.0, "evals": 0} for name in surrogates}
    for m in ids:
        V, F = host[m]
        Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
        grp = ranker._kmeans_groups(V, F, 8, seed=m)
        fitted, _ = api.fit(Vt, Ft, torch.from_numpy(grp).cuda(), 8)
        fitted = fitted.cpu().numpy()
        g = np.random.default_rng(m)
        cen = V.astype(np.float64)[F].mean(axis=1)
        init, bg = [], []
        for j in range(8):
            tris = np.nonzero(grp == j)[0]
            for t in g.choice(tris, size=min(4, len(tris)), replace=False):
                b = fitted[j].copy()
                b[:3] = cen[t]
                b[12:] = 0.0
                init.append(b)
                bg.append(j)
        vol, frame = api.occupancy_volume(Vt, Ft, nb=16, seed=1)
        for name, sur in surrogates.items():
            with api.Lloyd(Vt, Ft, R=64, seed=m, pops_per_round=32) as L:
                L.set_groups(grp, np.array(bg, np.int32), np.array(init, np.float32))
                if sur is not None:
                    L.set_surrogate(api.Surrogate(sur[0], vol, frame, verify_top=sur[1], max_error=0.05,
                                                  judge_every=32))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(2):
                    L.step()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                out = L.get()
            r = res[name]
            r["moves"] += out["counters"]["moves"]
            r["evals"] += out["counters"]["evals"]
            r["seconds"] += dt
            r["layer_error"] += out["layer_error"]
    for name, r in res.items():
        r["moves_per_s"] = r["moves"] / r["seconds"]
    for name, r in res.items():
        if name != "exact":
            r["speedup"] = r["moves_per_s"] / res["exact"]["moves_per_s"]
            r["e_ratio"] = r["layer_error"] / res["exact"]["layer_error"]
    return res


def surrogate_comparison(api, torch, Vt, Ft, hp, exact, judge_every=32):
    """Train the ranker on 1.05 M exact outer fractions of the batched workload's
    noisy spheres 0-223 (4,096 random boxes and 64 flood-candidate groups of 9
    boxes per mesh), validate on spheres 224-255 against the occupancy
    estimate, then: the torus hierarchy with network-ranked floods,
    occupancy-mean-ranked floods (the same machinery, network output 0) and
    network-ranked floods verifying the 4 best candidates per box; and two
    Lloyd iterations on 16 held-out spheres (240-255) under each mode."""
    from paper_2203_10521_amd import ranker
    host = config3_meshes()
    t0 = time.perf_counter()
    Xs, ts = [], []
    for m in range(224):
        X, t, *_ = ranker_eval_set(api, torch, *host[m], seed=100 + m, n_single=4096)
        Xs.append(X)
        ts.append(t)
    X, t = torch.cat(Xs), torch.cat(ts)
    del Xs, ts
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    P, losses = ranker.train(X, t, steps=3000, batch=4096, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    n_pairs = int(X.shape[0])
    del X, t
    val = ranker.summarise_metrics([ranker.ranking_metrics(P, *ranker_eval_set(api, torch, *host[m], seed=900 + m,
                                                                                 n_single=1024))
                                    for m in range(224, 256)])
    log(f"ranker validation: network MAE {val['network']['mae']:.5f} top-1 {val['network']['top1']:.3f}; "
        f"occupancy mean MAE {val['occupancy_mean']['mae']:.5f} top-1 {val['occupancy_mean']['top1']:.3f}")
    vol, frame = api.occupancy_volume(Vt, Ft, nb=16, seed=1)
    occ = ranker.occupancy_params()
    runs = {}
    for name, params, verify in (("network", P, 0), ("occupancy_mean", occ, 0), ("network_verify_top4", P, 4)):
        sur = api.Surrogate(params, vol, frame, verify_top=verify, max_error=0.05, judge_every=judge_every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = api.build_hierarchy(Vt, Ft, surrogate=sur, **hp)
        dt = time.perf_counter() - t1
        c = out["counters"]
        runs[name] = {"moves_per_s": c["moves"] / dt, "speedup": (c["moves"] / dt) / exact["moves_per_s"],
                      "final_e": float(out["e"][-1]), "e_ratio": float(out["e"][-1]) / exact["final_e"],
                      "exact_evals": c["evals"], "predictions": c["predicted"], "fallbacks": c["fallbacks"],
                      "build_s": dt}
        log(f"surrogate {name}: {runs[name]['speedup']:.2f}x exact moves/s, e ratio {runs[name]['e_ratio']:.4f}")
    held = lloyd_held_out(api, torch, host, range(240, 256),
                          {"exact": None, "network": (P, 0), "occupancy_mean": (occ, 0),
                           "network_verify_top4": (P, 4)})
    res = dict(runs["network"])
    res.update({"judge_every": judge_every, "exact_moves_per_s": exact["moves_per_s"],
                "exact_final_e": exact["final_e"], "exact_evals_without_ranker": exact["evals"],
                "occupancy_mean": runs["occupancy_mean"], "network_verify_top4": runs["network_verify_top4"],
                "held_out_config3_lloyd": held,
                "validation": val,
                "train": {"pairs": n_pairs, "steps": 3000, "batch": 4096, "data_s": data_s, "train_s": train_s,
                          "final_loss": losses[-1][1],
                          "data": "noisy spheres 0-223 of the batched workload (256 spheres, log-normal "
                                  "triangle counts); per sphere 4,096 random boxes around it + 64 flood-candidate "
                                  "groups (a base box and 8 one-triangle growths); validation: spheres 224-255"}})
    return res


def _oracle_box(args):
    from oracle import raygrid
    V, F, bx, R, seed, key = args
    return raygrid.raygrid_obv(V, F, bx[:3], bx[3:12].reshape(3, 3), bx[12:15], R, seed, key)["obv"]


def _exact_box(args):
    from oracle import exact
    V, F, bx = args
    return exact.obv(V, F, bx[:3], bx[3:12].reshape(3, 3), bx[12:15].astype(np.float64))


def _lscpu():
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:
        return None
    keep = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz")
    return {k.strip(): v.strip() for line in txt.splitlines() if ":" in line
            for k, v in [line.split(":", 1)] if k.strip() in keep}


def cpu_baseline(V, F, boxes, R, seed, budget_s=8.0):
    """The CPU oracle (float64 NumPy) on a bounded sample of the hierarchy's
    boxes: the discrete ray-grid oracle O1 in one process and in a pool of
    processes over boxes, and the exact clipped-prism oracle O2 in one process."""
    import multiprocessing as mp
    order = [b for b in [0, 1, 5, 21, 2, 6, 22, 40, 3, 7, 60, 84, 9, 30, 50, 70, 11, 33, 55, 77]
             if b < len(boxes) and np.all(boxes[b][12:] > 0)]
    done = 0
    t0 = time.perf_counter()
    for b in order:
        _oracle_box((V, F, boxes[b], R, seed, b))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    single = done / (time.perf_counter() - t0)
    cores = max(1, min(os.cpu_count() or 1, 16))
    sample = order[:min(len(order), 2 * cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_box, [(V, F, boxes[b], R, seed, b) for b in sample])
    pooled = len(sample) / (time.perf_counter() - t0)
    ex_done = 0
    t0 = time.perf_counter()
    for b in order:
        _exact_box((V, F, boxes[b]))
        ex_done += 1
        if time.perf_counter() - t0 > budget_s / 2:
            break
    exact_rate = ex_done / (time.perf_counter() - t0)
    return {"value": pooled, "unit": "box evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} boxes of the built torus hierarchy (layers 0-3, fixed order), R={R}, "
                      f"float64 NumPy ray-grid oracle (O1) in a pool of {cores} processes",
            "single_process": {"value": single, "boxes": done, "cores": 1},
            "exact_O2_single_process": {"value": exact_rate, "boxes": ex_done, "cores": 1,
                                        "kind": "exact clipped-prism oracle"},
            "os_cpu_count": os.cpu_count(), "lscpu": _lscpu()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-saturated", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the config 1 / 3 / 4 legs and the tree comparison")
    ap.add_argument("--judge-every", type=int, default=32, help="surrogate: every n-th ranked round is judged")
    ap.add_argument("--iters", type=int, default=HIER["iters"], help="Lloyd iterations per layer")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the memory-traffic counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        for _ in range(3):
            y = x.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "copies": 3, "ok": bool(y[0].item() == 1.0)}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is described in DESIGN.md and not run.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2203_10521_amd import api

    hp = dict(HIER, iters=args.iters)
    V, F = synth.noisy_torus(seed=SEED_MESH)
    Vt, Ft = torch.from_numpy(V).cuda(), torch.from_numpy(F).cuda()
    # create the library's scratch pools before the timed region
    api.outer_volume(Vt, Ft, torch.zeros((1, 15), dtype=torch.float32, device="cuda") + 0.5, 8)
    torch.cuda.synchronize()
    for w in range(args.warmup):
        api.build_hierarchy(Vt, Ft, **hp)
        log(f"warmup step {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    api.profile_enable(True)
    api.profile_read()
    evals = moves = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = api.build_hierarchy(Vt, Ft, **hp)
        evals += out["counters"]["evals"]
        moves += out["counters"]["moves"]
        log(f"timed step done: {out['counters']['evals']} evaluations")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cast_ms, launches, tests, nbytes, busy_ms = api.profile_read(busy=True)
    api.profile_enable(False)
    avg_ms, per_launch, tflops_launch, gbps_launch = kernel_rates(cast_ms, launches, tests, nbytes)
    # rates while the cast kernel runs: the launches of the two flood streams
    # overlap, so the tests are divided by the union of the launch intervals
    tflops = tests * FLOP_PER_TEST / (busy_ms * 1e-3) / 1e12 if busy_ms > 0 else 0.0
    gbps = nbytes / (busy_ms * 1e-3) / 1e9 if busy_ms > 0 else 0.0
    boxes_per_call = evals / max(launches, 1)
    algo_bytes = F.shape[0] * 36 + 68 * boxes_per_call

    result = {
        "metric": METRIC,
        "value": evals / dt,
        "unit": "box evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "noisy torus 65,536 triangles; hierarchy 1/4/16/64 boxes (4 layers, "
                               "branching 4); 20 Lloyd iterations per layer; 2 up/down sweeps; "
                               "128x128 rays per box face; K=32 pops per group per round",
                   "levels": hp["levels"], "branching": hp["branching"], "iters": hp["iters"],
                   "sweeps": hp["sweeps"], "R": hp["R"], "pops_per_round": hp["pops_per_round"],
                   "n_triangles": int(F.shape[0])},
        "evals_per_step": evals / args.steps,
        "moves_per_s": moves / dt,
        "hierarchy_error": out["e"].tolist(),
        "tests_per_s": tests / (busy_ms * 1e-3) if busy_ms > 0 else None,
        "cast_avg_ms": avg_ms,
        "cast_busy_ms_per_step": busy_ms / args.steps,
        "cast_sum_ms_per_step": cast_ms / args.steps,
        "cast_launches": launches,
        "tests_per_launch": per_launch,
        # the cast kernel's work is FP32 ray-triangle tests: 16 FLOP each, graded
        # against the FP32 vector peak (packed; the non-packed ceiling beside it)
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_PEAK_TFLOPS, "traffic": traffic_bytes(),
                     "kernel": "k_cast", "flop_per_test": FLOP_PER_TEST, "time": "union of launch intervals",
                     "achieved_per_launch": tflops_launch, "frac_per_launch": tflops_launch / FP32_PEAK_TFLOPS,
                     "peak_nonpacked": FP32_NONPACKED_TFLOPS, "frac_nonpacked": tflops / FP32_NONPACKED_TFLOPS},
        "hbm_traffic": (None if traffic_bytes() is None else
                        {"bytes_per_launch": traffic_bytes(), "ratio_to_algorithmic": traffic_bytes() / algo_bytes,
                         "gbps_at_cast_avg": traffic_bytes() / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None,
                         "source": "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"}),
        "culling_stream": {"bytes_per_launch": nbytes / max(launches, 1), "achieved_gbps": gbps,
                           "achieved_gbps_per_launch": gbps_launch,
                           "peak_gbps": HBM_PEAK_GBPS, "frac": gbps / HBM_PEAK_GBPS,
                           "algorithmic_bytes_per_launch": algo_bytes,
                           "ratio_to_algorithmic": (nbytes / max(launches, 1)) / algo_bytes,
                           "boxes_per_call": boxes_per_call},
    }
    log(f"hierarchy: {evals / dt:.0f} evals/s, cast {avg_ms:.4f} ms avg over {launches} launches")
    if not args.no_legs:
        log("tree comparison, config 1 / 3 / 4 legs")
        result["obb_tree"] = obb_tree_comparison(api, torch, Vt, Ft, out, hp)
        result["exact_evaluator"] = exact_evaluator_leg(api, torch, Vt, Ft, out["boxes"], hp["R"], hp["seed"])
        result["collision_queries"] = collision_leg(api, torch, V, Vt, Ft, out, hp)
        result["legs"] = {"config1": leg_config1(api, torch), "config3": leg_config3(api, torch),
                          "config4": leg_config4(api, torch)}
    if not args.no_surrogate:
        log("surrogate comparison: training the ranker, then the guided builds")
        result["surrogate"] = surrogate_comparison(
            api, torch, Vt, Ft, hp, {"moves_per_s": moves / dt, "final_e": float(out["e"][-1]),
                                     "evals": evals / args.steps}, judge_every=args.judge_every)
    if not args.no_saturated:
        log("saturated evaluation")
        result["saturated"] = saturated(api, torch, Vt, Ft, out["boxes"], hp["R"], hp["seed"])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(V, F, out["boxes"], hp["R"], hp["seed"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
