"""Canonical digests of a run's state and records, shared by the script that
writes the stored oracle values and by the GPU tests that compare with them.

Digests only (no method arithmetic): SHA-256 over little-endian bytes in a
fixed order, shortened to 16 hex digits.
"""
import hashlib

import numpy as np

INT_FIELDS = ["R_i", "sumE", "sumE2", "sumAbsM", "sumM2", "nPairs", "sumQ", "sumAbsQ", "sumQ2",
              "sumQl", "sumQl2", "famSumSq", "famMax", "nFam", "Emin", "status"]


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype.str).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()[:16]


def state_digests(spins, E, fam, counts) -> dict:
    """spins [R_i, N] int8 (+-1), energies and family labels [R_i] int32,
    descendant counts of the last resampling [R_{i-1}] int32."""
    return {"spins": digest(np.asarray(spins, np.int8)), "E": digest(np.asarray(E, np.int32)),
            "fam": digest(np.asarray(fam, np.int32)), "counts": digest(np.asarray(counts, np.int32))}


def record_digest(rec) -> str:
    """The integer fields of one record (R_i ... status), in a fixed order."""
    return digest(np.array([int(rec[f]) for f in INT_FIELDS], np.int64))
