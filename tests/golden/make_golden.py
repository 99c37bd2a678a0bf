"""Writes hth_golden.json: hash values of the frozen family computed by the
CPU oracle only (oracle/) on inputs from the seeded generators.

The paper prints no test vectors, so these values are self-generated: they
freeze the family as this repository defines it (code matrices, seed layout,
tree keys, tail and length terms).  Any change to them is a change of the
family and must name, in its commit message, the passage of the paper or the
reading of it that justifies it.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2104_08865_amd import workloads as wl  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hth_golden.json")


def cases():
    for b in (8, 4):
        for width in (16, 24, 32, 40):
            xb = wl.execution_bytes(width) * b // 8
            lens = [0, 1, 7, 8, 9, 63, 64, 100, 1024, xb - 8, xb - 1, xb, xb + 1, 8 * xb - 1, 8 * xb,
                    8 * xb + 1, 9 * xb + 17, 64 * xb - 1, 64 * xb, 64 * xb + 1, 65 * xb + 8 * xb + 3,
                    512 * xb + 5]
            for user_seed in (1, 0x0123456789ABCDEF):
                for n in lens:
                    yield b, user_seed, width, n


def composed_cases():
    for b in (8, 4):
        for width in (16, 24, 32, 40):
            xb = wl.execution_bytes(width) * b // 8
            for n in (0, 1, 8, width - 1, width, width + 1, 100, xb - 1, xb, 8 * xb + 3):
                yield b, 1, 2, width, n


def main():
    rows = []
    ents = {}
    for b, user_seed, width, n in cases():
        if (b, user_seed) not in ents:
            ents[(b, user_seed)] = oracle.expand_seed(user_seed, b=b)
        data = wl.random_bytes(1, n)
        h = oracle.hash_bytes(ents[(b, user_seed)], data.tobytes(), width, b=b)
        row = {"user_seed": user_seed, "width": width, "length": n, "bytes_seed": 1, "hash": bytes(h).hex()}
        if b != 8:
            row["block_words"] = b
        rows.append(row)
    composed = []
    for b, user_seed, tab_seed, width, n in composed_cases():
        if (b, user_seed) not in ents:
            ents[(b, user_seed)] = oracle.expand_seed(user_seed, b=b)
        data = wl.random_bytes(1, n)
        z = oracle.hash64(ents[(b, user_seed)], oracle.tab_expand(tab_seed, width), data.tobytes(), width, b=b)
        composed.append({"user_seed": user_seed, "tab_seed": tab_seed, "width": width, "length": n,
                         "bytes_seed": 1, "block_words": b, "hash64": f"{z:016x}"})
    doc = {
        "about": "HalftimeHash values of the frozen family, written by tests/golden/make_golden.py "
                 "from the CPU oracle; data = first `length` bytes of the splitmix64 byte buffer "
                 "with seed `bytes_seed`; entropy = splitmix64 expansion of `user_seed`; "
                 "`block_words` (default 8) is the family's block size b.  `composed`: the 64-bit "
                 "composition with simple tabulation (inner width `width`, tables = splitmix64 "
                 "expansion of `tab_seed`), as a hexadecimal integer.",
        "cases": rows,
        "composed": composed,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    print(f"wrote {len(rows)} cases and {len(composed)} composed cases to {OUT}")


if __name__ == "__main__":
    main()
