"""Python binding of libobbv: argument marshalling only.

Every function takes torch tensors on the HIP device (``cuda:0`` under ROCm),
checks dtypes and shapes, and calls the C entry point of the same name on the
current torch stream.  All arithmetic runs in the library's HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib

BOX_FLOATS = 15  # center[3], axes[9] (row k = local axis k), half[3]


class ObbvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libobbv error {code}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise ObbvError(code, _lib.lib().obbv_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name, shape_tail=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    return t


def mesh_struct(V, F):
    _dev(V, torch.float32, "vertices", (3,))
    _dev(F, torch.int32, "triangles", (3,))
    return _lib.ObbvMesh(V.data_ptr(), F.data_ptr(), V.shape[0], F.shape[0])


def version():
    return _lib.lib().obbv_version().decode()


def status(stream=None):
    flags = ctypes.c_uint32(0)
    _check(_lib.lib().obbv_status(_stream(stream), ctypes.byref(flags)))
    return flags.value


def release():
    _check(_lib.lib().obbv_release())


def validate_mesh(V, F, stream=None):
    """(code, report[4], volume) -- code 0 means a closed, outward oriented solid."""
    m = mesh_struct(V, F)
    rep = (ctypes.c_int32 * 4)()
    vol = ctypes.c_double(0.0)
    code = _lib.lib().obbv_validate_mesh(ctypes.byref(m), rep, ctypes.byref(vol), _stream(stream))
    return code, list(rep), vol.value


def _params(R, seed, axis_mask, block_rays):
    return _lib.ObbvOvParams(int(R), int(axis_mask), int(seed) & ((1 << 64) - 1), int(block_rays), 0)


def outer_volume(V, F, boxes, R, seed=0, axis_mask=7, block_rays=0, box_key=None, out=None, stream=None):
    """OBV of every box against the mesh (V, F); float64 tensor [n_boxes]."""
    return outer_volume_ex(V, F, boxes, R, seed, axis_mask, block_rays, box_key, out=out, stream=stream)["obv"]


def outer_volume_ex(V, F, boxes, R, seed=0, axis_mask=7, block_rays=0, box_key=None, rays=False,
                    out=None, stream=None, meshes=None, box_mesh=None):
    """Outer volume with the optional per-axis and per-ray outputs of obbv_outer_volume_ex.

    ``meshes`` (list of (V, F)) with ``box_mesh`` (int32 [n_boxes]) evaluates boxes
    against several meshes in one call; then V and F are ignored.
    """
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    n = boxes.shape[0]
    dev = boxes.device
    if meshes is None:
        meshes = [(V, F)]
    structs = (_lib.ObbvMesh * len(meshes))(*[mesh_struct(v, f) for v, f in meshes])
    if box_mesh is not None:
        _dev(box_mesh, torch.int32, "box_mesh")
    if box_key is not None:
        _dev(box_key, torch.int32, "box_key")
    obv = out if out is not None else torch.empty(n, dtype=torch.float64, device=dev)
    _dev(obv, torch.float64, "out")
    vin = torch.empty((n, 3), dtype=torch.float64, device=dev)
    side = torch.empty((n, 3), dtype=torch.int32, device=dev)
    rq = rh = None
    if rays:
        rq = torch.empty((n, 3, R, R), dtype=torch.int32, device=dev)
        rh = torch.empty((n, 3, R, R), dtype=torch.int32, device=dev)
    p = _params(R, seed, axis_mask, block_rays)
    _check(_lib.lib().obbv_outer_volume_ex(structs, len(meshes), _ptr(boxes), _ptr(box_mesh), _ptr(box_key),
                                           n, ctypes.byref(p), _ptr(obv), _ptr(vin), _ptr(rq), _ptr(rh),
                                           _ptr(side), _stream(stream)))
    return {"obv": obv, "vin_axis": vin, "ray_q": rq, "ray_hits": rh, "side": side}


def outer_volume_exact(V, F, boxes, axis=0, out=None, stream=None):
    """obbv_outer_volume_exact: exact OBV of every box along local axis `axis`
    (clipped-prism integral in float64); float64 tensor [n_boxes]."""
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    n = boxes.shape[0]
    m = mesh_struct(V, F)
    obv = out if out is not None else torch.empty(n, dtype=torch.float64, device=boxes.device)
    _dev(obv, torch.float64, "out")
    _check(_lib.lib().obbv_outer_volume_exact(ctypes.byref(m), _ptr(boxes), n, int(axis), _ptr(obv),
                                              _stream(stream)))
    return obv


def outer_volume_central(V, F, boxes, m, out=None, stream=None):
    """obbv_outer_volume_central: the central-projection estimate of every box's
    OBV with a 6 x m x m cube map; float64 tensor [n_boxes]."""
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    n = boxes.shape[0]
    mm = mesh_struct(V, F)
    obv = out if out is not None else torch.empty(n, dtype=torch.float64, device=boxes.device)
    _dev(obv, torch.float64, "out")
    _check(_lib.lib().obbv_outer_volume_central(ctypes.byref(mm), _ptr(boxes), n, int(m), _ptr(obv),
                                                _stream(stream)))
    return obv


def collision_queries(nodes, levels, branching, spheres, node_used=None, stream=None):
    """obbv_collision_queries: (tests, hits) int32 tensors [n_spheres] of sphere
    queries descending a level-order box hierarchy."""
    _dev(nodes, torch.float32, "nodes", (BOX_FLOATS,))
    _dev(spheres, torch.float32, "spheres", (4,))
    n_nodes = sum(int(branching) ** lv for lv in range(int(levels)))
    if nodes.shape[0] != n_nodes:
        raise ValueError(f"nodes must hold the {n_nodes} nodes of {levels} levels of branching {branching}")
    if node_used is not None:
        _dev(node_used, torch.uint8, "node_used")
        if node_used.shape != (n_nodes,):
            raise ValueError(f"node_used must have shape [{n_nodes}]")
    n = spheres.shape[0]
    tests = torch.empty(n, dtype=torch.int32, device=spheres.device)
    hits = torch.empty(n, dtype=torch.int32, device=spheres.device)
    _check(_lib.lib().obbv_collision_queries(_ptr(nodes), _ptr(node_used), int(levels), int(branching),
                                             _ptr(spheres), n, _ptr(tests), _ptr(hits), _stream(stream)))
    return tests, hits


def outer_volume_noalloc(V, F, boxes, R, seed=0, axis_mask=7, block_rays=0, box_key=None, out=None, status=None,
                         stream=None):
    """obbv_outer_volume_noalloc: OBV of every box with the library's fixed
    scratch array (no device allocation in the call); float64 [n_boxes]."""
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    m = mesh_struct(V, F)
    if box_key is not None:
        _dev(box_key, torch.int32, "box_key")
    if status is not None:
        _dev(status, torch.int32, "status")
    obv = out if out is not None else torch.empty(boxes.shape[0], dtype=torch.float64, device=boxes.device)
    _dev(obv, torch.float64, "out")
    p = _params(R, seed, axis_mask, block_rays)
    _check(_lib.lib().obbv_outer_volume_noalloc(ctypes.byref(m), _ptr(boxes), _ptr(box_key), boxes.shape[0],
                                                ctypes.byref(p), _ptr(obv), _ptr(status), _stream(stream)))
    return obv


def outer_volume_grouped(V, F, boxes, R, frames, box_frame, seed=0, axis_mask=7, block_rays=0, box_key=None,
                         out=None, stream=None):
    """obbv_outer_volume_grouped: boxes in groups sharing a centre and axes;
    frames [n_frames, 15] are the groups' unions, box_frame [n_boxes] int32."""
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    _dev(frames, torch.float32, "frames", (BOX_FLOATS,))
    _dev(box_frame, torch.int32, "box_frame")
    if box_key is not None:
        _dev(box_key, torch.int32, "box_key")
    n = boxes.shape[0]
    obv = out if out is not None else torch.empty(n, dtype=torch.float64, device=boxes.device)
    _dev(obv, torch.float64, "out")
    m = mesh_struct(V, F)
    p = _params(R, seed, axis_mask, block_rays)
    _check(_lib.lib().obbv_outer_volume_grouped(ctypes.byref(m), _ptr(boxes), _ptr(box_key), n, ctypes.byref(p),
                                                _ptr(frames), _ptr(box_frame), frames.shape[0], _ptr(obv),
                                                _stream(stream)))
    return obv


def outer_volume_raw(meshes_struct, n_meshes, boxes, box_mesh, box_key, n, params, out, stream=None):
    """Direct obbv_outer_volume call on prepared structs (used by the timing loop)."""
    _check(_lib.lib().obbv_outer_volume(meshes_struct, n_meshes, _ptr(boxes), _ptr(box_mesh), _ptr(box_key),
                                        n, ctypes.byref(params), _ptr(out), _stream(stream)))


def fit(V, F, tri_cluster, n_clusters, stream=None):
    """Covariance OBB per cluster: (boxes float32 [n, 15], eigenvalues float64 [n, 3])."""
    m = mesh_struct(V, F)
    _dev(tri_cluster, torch.int32, "tri_cluster")
    if tri_cluster.shape[0] != F.shape[0]:
        raise ValueError("tri_cluster needs one entry per triangle")
    boxes = torch.empty((n_clusters, BOX_FLOATS), dtype=torch.float32, device=V.device)
    eig = torch.empty((n_clusters, 3), dtype=torch.float64, device=V.device)
    _check(_lib.lib().obbv_fit(ctypes.byref(m), _ptr(tri_cluster), int(n_clusters), _ptr(boxes), _ptr(eig),
                               _stream(stream)))
    return boxes, eig


def profile_enable(enable=True):
    """Record HIP events around every later ray-test kernel launch (and count its
    tests and the bytes it must read)."""
    _check(_lib.lib().obbv_profile_enable(1 if enable else 0))


def profile_read(busy=False):
    """(total ray-test milliseconds, launches, ray-triangle tests, algorithmic
    bytes read) since the last read; with busy=True a fifth value, the
    milliseconds during which at least one ray-test launch ran (launches on
    several streams overlap)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    t = ctypes.c_int64(0)
    b = ctypes.c_int64(0)
    u = ctypes.c_double(0.0)
    _check(_lib.lib().obbv_profile_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(t), ctypes.byref(b),
                                        ctypes.byref(u)))
    return (ms.value, n.value, t.value, b.value, u.value) if busy else (ms.value, n.value, t.value, b.value)


def _host_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


class Lloyd:
    """Same-layer Lloyd clustering state (obbv_lloyd_*); host arrays are numpy."""

    def __init__(self, V, F, R, seed=0, pops_per_round=32, delta=0.02, block_rays=0, stream=None):
        self._mesh = mesh_struct(V, F)
        self._keep = (V, F)
        self.n_triangles = F.shape[0]
        p = _lib.ObbvLloydParams(int(R), int(block_rays), int(seed) & ((1 << 64) - 1), int(pops_per_round), 0,
                                 float(delta))
        self._h = ctypes.c_void_p(0)
        _check(_lib.lib().obbv_lloyd_create(ctypes.byref(self._mesh), ctypes.byref(p), ctypes.byref(self._h)))
        self.n_boxes = 0
        self._stream = stream

    def set_groups(self, tri_group, box_group, boxes, box_slot=None):
        tri_group = np.ascontiguousarray(tri_group, dtype=np.int32)
        box_group = np.ascontiguousarray(box_group, dtype=np.int32)
        boxes = np.ascontiguousarray(boxes, dtype=np.float32).reshape(-1, BOX_FLOATS)
        slot = None if box_slot is None else np.ascontiguousarray(box_slot, dtype=np.uint32)
        self.n_boxes = boxes.shape[0]
        self.n_groups = int(box_group.max()) + 1 if len(box_group) else 0
        _check(_lib.lib().obbv_lloyd_set_groups(self._h, self.n_boxes, _host_ptr(tri_group), _host_ptr(box_group),
                                                _host_ptr(boxes), _host_ptr(slot)))

    def step(self):
        _check(_lib.lib().obbv_lloyd_step(self._h, _stream(self._stream)))

    def adjust(self):
        """One adjustment of every group (obbv_lloyd_adjust): per group 1 kept,
        0 undone, -1 not adjusted."""
        acc = np.empty(self.n_groups, np.int32)
        _check(_lib.lib().obbv_lloyd_adjust(self._h, _host_ptr(acc), _stream(self._stream)))
        return acc

    def get(self):
        tri_box = np.empty(self.n_triangles, np.int32)
        boxes = np.empty((self.n_boxes, BOX_FLOATS), np.float32)
        obv = np.empty(self.n_boxes, np.float64)
        e = ctypes.c_double(0.0)
        cnt = (ctypes.c_int64 * 6)()
        _check(_lib.lib().obbv_lloyd_get(self._h, _host_ptr(tri_box), _host_ptr(boxes), _host_ptr(obv),
                                         ctypes.byref(e), cnt))
        return {"tri_box": tri_box, "boxes": boxes, "obv": obv, "layer_error": e.value,
                "counters": dict(zip(COUNTERS, list(cnt)))}

    def set_surrogate(self, surrogate):
        """A Surrogate (or None for exact evaluation of every candidate)."""
        self._sur = surrogate
        _check(_lib.lib().obbv_lloyd_set_surrogate(
            self._h, ctypes.byref(surrogate.struct()) if surrogate is not None else None))

    def record(self, cap):
        """Keep a uniform sample of up to cap evaluated (box, outer volume) pairs."""
        _check(_lib.lib().obbv_lloyd_record(self._h, int(cap)))
        self._rec_cap = int(cap)

    def take_records(self):
        """(boxes float32 [n, 15], obv float64 [n]) of the sample; clears it."""
        cap = getattr(self, "_rec_cap", 0)
        boxes = np.empty((max(cap, 1), BOX_FLOATS), np.float32)
        obv = np.empty(max(cap, 1), np.float64)
        n = ctypes.c_int64(0)
        _check(_lib.lib().obbv_lloyd_take_records(self._h, cap, _host_ptr(boxes), _host_ptr(obv), ctypes.byref(n)))
        return boxes[:n.value].copy(), obv[:n.value].copy()

    def close(self):
        if self._h:
            _lib.lib().obbv_lloyd_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


COUNTERS = ("evals", "rounds", "trivial", "moves", "predicted", "fallbacks")


class Surrogate:
    """Device arrays of a trained ranker (obbv_surrogate)."""

    def __init__(self, mlp_params, volume, frame, verify_top=0, max_error=0.05, judge_every=16):
        self.mlp_params, self.volume, self.frame = mlp_params, volume, frame
        self.verify_top, self.max_error, self.judge_every = int(verify_top), float(max_error), int(judge_every)

    def struct(self):
        self._s = _lib.ObbvSurrogate(self.mlp_params.data_ptr(), self.volume.data_ptr(), self.frame.data_ptr(),
                                     self.volume.shape[0], self.verify_top, self.max_error, self.judge_every)
        return self._s


def build_obb_tree(V, F, levels, branching, stream=None):
    """obbv_build_obb_tree: the top-down covariance-box tree (numpy outputs)."""
    m = mesh_struct(V, F)
    n_nodes = sum(branching ** l for l in range(levels))
    nt = F.shape[0]
    boxes = np.empty((n_nodes, BOX_FLOATS), np.float32)
    parent = np.empty(n_nodes, np.int32)
    tri_node = np.empty((levels, nt), np.int32)
    _check(_lib.lib().obbv_build_obb_tree(ctypes.byref(m), int(levels), int(branching), _host_ptr(boxes),
                                          _host_ptr(parent), _host_ptr(tri_node), _stream(stream)))
    return {"boxes": boxes, "parent": parent, "tri_node": tri_node}


def build_hierarchy(V, F, levels, branching, iters, sweeps, R, seed=0, pops_per_round=32, delta=0.02, block_rays=0,
                    surrogate=None, stream=None):
    """obbv_build_hierarchy; returns numpy outputs (boxes, obv, parent, tri_node, e, counters)."""
    m = mesh_struct(V, F)
    sp = ctypes.pointer(surrogate.struct()) if surrogate is not None else None
    p = _lib.ObbvHierParams(int(levels), int(branching), int(iters), int(sweeps), int(R), int(block_rays),
                            int(pops_per_round), 0, int(seed) & ((1 << 64) - 1), float(delta), sp)
    n_nodes = sum(branching ** level for level in range(levels))
    nt = F.shape[0]
    boxes = np.zeros((n_nodes, BOX_FLOATS), np.float32)
    obv = np.zeros(n_nodes, np.float64)
    parent = np.zeros(n_nodes, np.int32)
    tri_node = np.zeros((levels, nt), np.int32)
    e = np.zeros(1 + sweeps, np.float64)
    cnt = np.zeros(6, np.int64)
    _check(_lib.lib().obbv_build_hierarchy(ctypes.byref(m), ctypes.byref(p), _host_ptr(boxes), _host_ptr(obv),
                                           _host_ptr(parent), _host_ptr(tri_node), _host_ptr(e), _host_ptr(cnt),
                                           _stream(stream)))
    return {"boxes": boxes, "obv": obv, "parent": parent, "tri_node": tri_node, "e": e,
            "counters": dict(zip(COUNTERS, cnt.tolist()))}


def mesh_frame(V):
    """[4] float32: bounding-box centre xyz and diagonal of a vertex tensor."""
    lo = V.min(dim=0).values
    hi = V.max(dim=0).values
    return torch.cat([(lo + hi) / 2, torch.linalg.norm(hi - lo).reshape(1)]).to(torch.float32).contiguous()


def box_features(boxes, seed=0, meshes=None, box_mesh=None, frames=None, stream=None):
    """[n, 544] float32 ranker inputs (obbv_box_features)."""
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    n = boxes.shape[0]
    structs = (_lib.ObbvMesh * len(meshes))(*[mesh_struct(v, f) for v, f in meshes])
    if frames is None:
        frames = torch.stack([mesh_frame(v) for v, _ in meshes]).contiguous()
    _dev(frames, torch.float32, "frames", (4,))
    if box_mesh is not None:
        _dev(box_mesh, torch.int32, "box_mesh")
    X = torch.empty((n, 544), dtype=torch.float32, device=boxes.device)
    _check(_lib.lib().obbv_box_features(structs, len(meshes), _ptr(boxes), _ptr(box_mesh), n, _ptr(frames),
                                        int(seed) & ((1 << 64) - 1), _ptr(X), _stream(stream)))
    return X


def mlp_param_count():
    return int(_lib.lib().obbv_mlp_param_count())


def mlp_pack(p):
    """Pack a dict of numpy parameters (W1, b1, W2, b2, w3, b3) into the float32 vector."""
    return np.concatenate([np.asarray(p[k], np.float64).reshape(-1) for k in ("W1", "b1", "W2", "b2", "w3", "b3")]
                          ).astype(np.float32)


def mlp_unpack(v):
    v = np.asarray(v, np.float64)
    sizes = [("W1", (544, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)), ("w3", (256,)), ("b3", (1,))]
    out, o = {}, 0
    for k, shp in sizes:
        n = int(np.prod(shp))
        out[k] = v[o:o + n].reshape(shp)
        o += n
    return out


def mlp_forward(params, X, stream=None):
    _dev(params, torch.float32, "params")
    _dev(X, torch.float32, "X", (544,))
    f = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(_lib.lib().obbv_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(f), _stream(stream)))
    return f


def mlp_train_step(params, m, v, step, X, target, lr, want_grad=False, stream=None):
    """One Adam step in place; returns (loss tensor [1], gradient tensor or None)."""
    for t, name in ((params, "params"), (m, "adam_m"), (v, "adam_v"), (target, "target")):
        _dev(t, torch.float32, name)
    _dev(X, torch.float32, "X", (544,))
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    grad = torch.empty_like(params) if want_grad else None
    _check(_lib.lib().obbv_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), int(step), _ptr(X), _ptr(target),
                                          X.shape[0], float(lr), _ptr(loss), _ptr(grad), _stream(stream)))
    return loss, grad


def volume_frame(V, nb, margin=0.02):
    """[10] float32 frame of an occupancy volume: origin xyz, voxel size xyz (the
    bounding box grown by `margin` of its diagonal), bounding-box centre, diagonal."""
    lo = V.min(dim=0).values.double()
    hi = V.max(dim=0).values.double()
    diag = torch.linalg.norm(hi - lo)
    lo2, hi2 = lo - margin * diag, hi + margin * diag
    vox = (hi2 - lo2) / (8 * nb)
    return torch.cat([lo2, vox, (lo + hi) / 2, diag.reshape(1)]).to(torch.float32).contiguous()


def occupancy_volume(V, F, nb=16, seed=0, frame=None, stream=None):
    """(volume [8nb, 8nb, 8nb] float32 indexed [z, y, x], frame [10])."""
    m = mesh_struct(V, F)
    if frame is None:
        frame = volume_frame(V, nb)
    N = 8 * nb
    vol = torch.empty((N, N, N), dtype=torch.float32, device=V.device)
    _check(_lib.lib().obbv_occupancy_volume(ctypes.byref(m), int(nb), _ptr(frame), int(seed) & ((1 << 64) - 1),
                                            _ptr(vol), _stream(stream)))
    return vol, frame


def sample_features(volume, frame, boxes, stream=None):
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    X = torch.empty((boxes.shape[0], 544), dtype=torch.float32, device=boxes.device)
    _check(_lib.lib().obbv_sample_features(_ptr(volume), volume.shape[0], _ptr(frame), _ptr(boxes), boxes.shape[0],
                                           _ptr(X), _stream(stream)))
    return X



def mlp_rank_boxes(params, volume, frame, boxes, stream=None):
    """Predicted outer fractions of `boxes` [n, 15] in one launch (inputs sampled
    from `volume` on chip); the same bits as mlp_forward(sample_features(...))."""
    _dev(params, torch.float32, "params")
    _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
    f = torch.empty(boxes.shape[0], dtype=torch.float32, device=boxes.device)
    _check(_lib.lib().obbv_mlp_rank_boxes(_ptr(params), _ptr(volume), volume.shape[0], _ptr(frame), _ptr(boxes),
                                          boxes.shape[0], _ptr(f), _stream(stream)))
    return f

class OuterVolumePlan:
    """obbv_ov_plan_*: an autotuned, graph-captured evaluation of fixed arrays."""

    def __init__(self, boxes, R, seed=0, axis_mask=7, block_rays=0, meshes=None, box_mesh=None, box_key=None,
                 headroom=1.25, stream=None):
        _dev(boxes, torch.float32, "boxes", (BOX_FLOATS,))
        self.boxes, self.box_mesh, self.box_key, self._meshes = boxes, box_mesh, box_key, meshes
        self._structs = (_lib.ObbvMesh * len(meshes))(*[mesh_struct(v, f) for v, f in meshes])
        self.out = torch.empty(boxes.shape[0], dtype=torch.float64, device=boxes.device)
        self._p = _params(R, seed, axis_mask, block_rays)
        self._h = ctypes.c_void_p(0)
        _check(_lib.lib().obbv_ov_plan_create(self._structs, len(meshes), _ptr(boxes), _ptr(box_mesh),
                                              _ptr(box_key), boxes.shape[0], ctypes.byref(self._p), _ptr(self.out),
                                              float(headroom), _stream(stream), ctypes.byref(self._h)))

    def launch(self, stream=None):
        _check(_lib.lib().obbv_ov_plan_launch(self._h, _stream(stream)))
        return self.out

    def info(self):
        block_rays = ctypes.c_int32(0)
        caps = (ctypes.c_int64 * 3)()
        tms = (ctypes.c_float * 3)()
        _check(_lib.lib().obbv_ov_plan_info(self._h, ctypes.byref(block_rays), caps, tms))
        return {"block_rays": block_rays.value, "caps": list(caps), "tuned_ms": list(tms)}

    def close(self):
        if self._h:
            _lib.lib().obbv_ov_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
