"""Oracle values stored under ``tests/golden/`` (written by
``tests/golden/make_oracle_fixtures.py``, which calls only the oracle)."""
import hashlib
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def input_hash(*arrays) -> str:
    """SHA-256 over the FP64 bytes of the generated inputs."""
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def load(name: str, *inputs):
    """The stored fixture ``name``; when ``inputs`` are given, their hash
    must equal the one recorded with the fixture."""
    d = dict(np.load(os.path.join(GOLDEN, name + ".npz")))
    if inputs:
        assert str(d["hash"]) == input_hash(*inputs), f"{name}: inputs differ from the fixture's"
    return d
