"""The oracle still produces the frozen values in tests/golden/hth_golden.json
(written by tests/golden/make_golden.py from the oracle alone)."""
import json
import os

from paper_2104_08865_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hth_golden.json")


def test_oracle_matches_golden(oracle_lib):
    doc = json.load(open(GOLDEN))
    ents = {}
    for row in doc["cases"]:
        s, b = row["user_seed"], row.get("block_words", 8)
        if (s, b) not in ents:
            ents[(s, b)] = oracle_lib.expand_seed(s, b=b)
        data = wl.random_bytes(row["bytes_seed"], row["length"])
        h = oracle_lib.hash_bytes(ents[(s, b)], data.tobytes(), row["width"], b=b)
        assert bytes(h).hex() == row["hash"], row


def test_oracle_matches_golden_composed(oracle_lib):
    doc = json.load(open(GOLDEN))
    assert len(doc["composed"]) == 80
    for row in doc["composed"]:
        ent = oracle_lib.expand_seed(row["user_seed"], b=row["block_words"])
        tab = oracle_lib.tab_expand(row["tab_seed"], row["width"])
        data = wl.random_bytes(row["bytes_seed"], row["length"])
        z = oracle_lib.hash64(ent, tab, data.tobytes(), row["width"], b=row["block_words"])
        assert f"{z:016x}" == row["hash64"], row
