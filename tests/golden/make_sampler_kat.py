"""Writes sampler_kat.json: known-answer index sets from the oracle sampler.

Calls only oracle/.  Run from the repository root:
    python tests/golden/make_sampler_kat.py
The library's own sampler is checked against this file bit for bit.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.sampler import draw_sample  # noqa: E402

CASES = [
    # seed, t, dims, I sizes, J sizes (None = chidori)
    (0, 0, [100, 100, 100], [42, 42, 42], None),
    (0, 3, [100, 100, 100], [42, 42, 42], [83, 83, 83]),
    (7, 0, [300, 300, 300], [86, 86, 86], [172, 172, 172]),
    (123456789, 11, [240, 320, 3, 400], [110, 116, 3, 60], [120, 130, 5, 140]),
    (2**64 - 1, 2, [5, 7], [5, 3], [7, 4]),
    (42, 1, [20, 20, 20], [18, 18, 18], [324, 324, 324]),
]


def main():
    out = []
    for seed, t, dims, I_sz, J_sz in CASES:
        s = draw_sample(seed, t, dims, I_sz, J_sz)
        out.append({
            "seed": seed, "t": t, "dims": dims, "I_sizes": I_sz,
            "J_sizes": J_sz,
            "I": [list(map(int, x)) for x in s.I],
            "J_cols": [list(map(int, x)) for x in s.J_cols] if J_sz else None,
        })
    with open(os.path.join(HERE, "sampler_kat.json"), "w") as f:
        f.write("[\n" + ",\n".join(json.dumps(c) for c in out) + "\n]\n")


if __name__ == "__main__":
    main()
