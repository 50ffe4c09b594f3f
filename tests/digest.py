"""Per-generation digests used to compare whole runs (test infrastructure only).

A digest is the SHA-256 of the observables of one generation in a fixed order and dtype:
labels (int32, rows in selection order) when present, A and S (int64), the bit patterns of
f1 and f2 (float64), and, from generation 1 on, rank (int32) and crowding distance bits.
"""
import hashlib

import numpy as np


def state_digest(labels, A, S, f1, f2, rank, crowd, with_labels=True) -> str:
    h = hashlib.sha256()
    if with_labels:
        h.update(np.ascontiguousarray(labels, dtype=np.int32).tobytes())
    h.update(np.ascontiguousarray(A, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(S, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(f1, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(f2, dtype=np.float64).tobytes())
    if rank is not None:
        h.update(np.ascontiguousarray(rank, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(crowd, dtype=np.float64).tobytes())
    return h.hexdigest()[:32]


def front_digest(labels, A, S, f1, f2, selected) -> str:
    h = hashlib.sha256()
    for a, dt in [(labels, np.int32), (A, np.int64), (S, np.int64), (f1, np.float64),
                  (f2, np.float64)]:
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    h.update(np.int64(selected).tobytes())
    return h.hexdigest()[:32]
