"""The oracle run over host processes, for GPU tests whose oracle side would
take minutes in one process (every stream of the 256-image batch, thousands
of exhaustive-search ranges).

Workers start with the spawn method and import numpy and the oracle only,
never the GPU runtime, and each keeps its BLAS to one thread.  At most 16
workers: one GPU's share of the host.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

_LIMITS = None


def workers() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _init():
    global _LIMITS
    from threadpoolctl import threadpool_limits
    _LIMITS = threadpool_limits(limits=1)


def _encode(args):
    from oracle import mns
    img, b_max, b_min, thr = args
    return mns.encode(img, b_max, b_min, list(thr))


def _best(args):
    from oracle import fullsearch
    img, xs, ys, B = args
    return fullsearch.best_matches(img, xs, ys, B)


def pool() -> ProcessPoolExecutor:
    return ProcessPoolExecutor(workers(), mp_context=mp.get_context("spawn"), initializer=_init)


def encode_all(ex, images, b_max, b_min, thr):
    """Futures of the oracle's streams, one per image."""
    return [ex.submit(_encode, (img, b_max, b_min, tuple(thr))) for img in images]


def best_matches(ex, img, xs, ys, B, per_task: int = 32):
    """Futures of fullsearch.best_matches over consecutive slices of the
    ranges (xs, ys), per_task ranges each."""
    return [ex.submit(_best, (img, xs[s:s + per_task], ys[s:s + per_task], B))
            for s in range(0, len(xs), per_task)]
