"""The test-side 64-bit FNV-1a (used to check octax_digest) against the
published FNV reference values, and the oracle-state conversion it hashes
against the library's own record layout."""
import numpy as np

from tests.golden_util import GOLDEN
from tests.parity_util import fnv1a64, oracle_env_state_bytes


def test_fnv1a64_reference_values():
    for line in open(f"{GOLDEN}/fnv1a64.txt"):
        if line.startswith("#") or "|" not in line:
            continue
        text, want = line.rstrip("\n").rsplit("|", 1)
        data = np.frombuffer(text.strip().encode(), dtype=np.uint8).reshape(1, -1)
        assert int(fnv1a64(data)[0]) == int(want.strip(), 16), text


def test_oracle_state_record_matches_the_oracle():
    from oracle import oracle as O
    from paper_2510_01764_amd import workload as W
    spec = W.make_config("c1")
    b = O.OracleBatch(spec)
    for k in range(30):
        b.step(spec.actions(k, 1)[0], want_obs=False)
    st = b.get_state()
    rec = oracle_env_state_bytes(st)
    assert rec.dtype.itemsize == 5192
    for e in range(len(st)):
        for y in range(32):
            row = int(rec["fb"][e, y])
            assert [(row >> (63 - x)) & 1 for x in range(64)] == list(st["disp"][e, y])
    assert np.array_equal(rec["ram"], st["mem"]) and np.array_equal(rec["v"], st["v"])
