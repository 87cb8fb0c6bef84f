"""Writes tests/golden/tiny_oracle.txt: oracle values for the 80-atom H2/Pt(111) cell.

Calls only the FP64 oracle and the seeded input generator. Rerun after a change to
the oracle's arithmetic that a passage of the paper justifies:
    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import evaluate as ev  # noqa: E402
from oracle.hyper import DEFAULT  # noqa: E402
from paper_2204_12573_amd import structures as S  # noqa: E402

ATOMS = [0, 15, 31, 48, 63, 64, 67, 70, 75, 79]


def main():
    st = S.config_tiny()
    beta, gamma = S.random_model(DEFAULT.n_desc)
    r = ev.evaluate(st.pos, st.species, st.box, beta, gamma)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_oracle.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle on the 80-atom cell (4x4x4 Pt(111) + 8 H2, seed 0), random PSD\n")
        f.write("# beta/Sigma (seeds 1..4, scale 1e-3). Written by tests/golden/make_golden.py.\n")
        f.write(f"E_total {r.energy!r}\n")
        f.write("# atom species e sigma fx fy fz\n")
        for a in ATOMS:
            f.write(f"{a} {st.species[a]} {float(r.e[a])!r} {float(r.sigma[a])!r} {float(r.f[a,0])!r} {float(r.f[a,1])!r} {float(r.f[a,2])!r}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
