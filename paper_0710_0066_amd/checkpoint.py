"""Checkpoint and resume of an HMC run: host-side I/O only, no arithmetic of the method.

A checkpoint holds the canonical FP64 gauge field (complex128, [V][4][3][3]), the
trajectory counter, and the state of the host random generator that draws the momenta,
the pseudo-fermion noise and the Metropolis numbers, so that a resumed run continues
bit for bit. It is one .npz file, written to a temporary name and renamed into place.
"""
import json
import os

import numpy as np


def save(path, U, trajectory, rng, extra=None):
    """U: canonical gauge field (torch tensor on any device, or numpy array); rng: a
    numpy Generator; extra: JSON-serialisable user data."""
    Uh = U.detach().cpu().numpy() if hasattr(U, "detach") else np.asarray(U)
    meta = {"trajectory": int(trajectory), "rng": rng.bit_generator.state, "extra": extra or {}}
    blob = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    tmp = str(path) + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, U=Uh, meta=blob)
    os.replace(tmp, path)


def load(path):
    """Returns (U as a numpy array, trajectory counter, numpy Generator, extra)."""
    with np.load(path, allow_pickle=False) as z:
        U = z["U"]
        meta = json.loads(bytes(z["meta"]).decode())
    state = meta["rng"]
    rng = np.random.Generator(getattr(np.random, state["bit_generator"])())
    rng.bit_generator.state = state
    return U, meta["trajectory"], rng, meta["extra"]
