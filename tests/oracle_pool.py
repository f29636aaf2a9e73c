"""The ray-grid oracle as an evaluator callable, on a pool of CPU processes.

Test infrastructure: a flood round asks for up to K x (boxes per group)
outer volumes at once, which the pool computes in parallel.  The workers are
started fresh (spawn) and never touch a GPU; each holds its own copy of the mesh.
"""
import multiprocessing as mp
import os

import numpy as np

from oracle import raygrid

_MESH = {}


def _init(V, F, R, seed):
    _MESH["args"] = (V, F, R, seed)


def _one(item):
    V, F, R, seed = _MESH["args"]
    slot, c, Q, h = item
    return raygrid.raygrid_obv(V, F, c, Q, h, R, seed, int(slot))["obv"]


class RaygridPool:
    def __init__(self, V, F, R, seed, workers=None):
        self.args = (np.asarray(V), np.asarray(F), int(R), int(seed))
        self.workers = workers or max(1, min(8, (os.cpu_count() or 1)))
        self.pool = None

    def __enter__(self):
        if self.workers > 1:
            self.pool = mp.get_context("spawn").Pool(self.workers, initializer=_init, initargs=self.args)
        else:
            _init(*self.args)
        return self

    def __exit__(self, *exc):
        if self.pool is not None:
            self.pool.terminate()
            self.pool.join()

    def __call__(self, items):
        items = [(int(s), np.asarray(c), np.asarray(Q), np.asarray(h)) for s, c, Q, h in items]
        if self.pool is None or len(items) < 4:
            if self.pool is None:
                return [_one(x) for x in items]
            return [raygrid.raygrid_obv(self.args[0], self.args[1], c, Q, h, self.args[2], self.args[3],
                                        s)["obv"] for s, c, Q, h in items]
        chunk = max(1, len(items) // (2 * self.workers))
        return self.pool.map(_one, items, chunksize=chunk)
