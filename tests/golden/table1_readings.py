"""Test 1.1 (Section 5.1, Table 1) under the readings the paper leaves open.

Runs the oracle's Test 1.1 (two-dimensional Maxwell molecules, BKW datum, 8 angles,
explicit Euler to t = 10, the printed boxes) for each reading in READINGS and prints a
markdown table of the relative L1 / L2 errors at 8^2, 16^2 and 32^2 beside the printed
ones.  Only ``oracle/`` is called.  Usage: ``python tests/golden/table1_readings.py``
(about half a minute).
"""
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.fks_oracle2d as O2  # noqa: E402

R_DEFAULT = 2.0 / (3.0 + math.sqrt(2.0))    # R / T
# (label, R / T, node offset, Nyquist modes zeroed, dt, projection)
READINGS = [
    ("node grid, R = 2T/(3+sqrt2), Nyquist zeroed, dt 0.02 (library default)", R_DEFAULT, 0.0, True, 0.02, True),
    ("same, dt 0.005", R_DEFAULT, 0.0, True, 0.005, True),
    ("same, no projection", R_DEFAULT, 0.0, True, 0.02, False),
    ("same, A = 16 angles", R_DEFAULT, 0.0, True, 0.02, True, 16),
    ("node grid, R = T/(2+sqrt2)", 1.0 / (2.0 + math.sqrt(2.0)), 0.0, True, 0.02, True),
    ("node grid, R = T/2", 0.5, 0.0, True, 0.02, True),
    ("node grid, R = 2T/(2+sqrt2)", 2.0 / (2.0 + math.sqrt(2.0)), 0.0, True, 0.02, True),
    ("node grid, Nyquist kept", R_DEFAULT, 0.0, False, 0.02, True),
    ("node grid, Nyquist kept, R = 2T/(2+sqrt2)", 2.0 / (2.0 + math.sqrt(2.0)), 0.0, False, 0.02, True),
    ("node grid, Nyquist kept, R = T/sqrt2", 1.0 / math.sqrt(2.0), 0.0, False, 0.02, True),
    ("node grid, Nyquist kept, R = T/sqrt2, dt 0.01", 1.0 / math.sqrt(2.0), 0.0, False, 0.01, True),
    ("cell centres, R = 2T/(3+sqrt2)", R_DEFAULT, 0.5, True, 0.02, True),
    ("cell centres, R = T/sqrt2, dt 0.02 (printed dt)", 1.0 / math.sqrt(2.0), 0.5, True, 0.02, True),
    ("cell centres, R = T/sqrt2, dt 0.01 (asserted reading)", 1.0 / math.sqrt(2.0), 0.5, True, 0.01, True),
]


def golden():
    rows = {}
    with open(os.path.join(HERE, "table1_test11_bkw2d.txt")) as fp:
        for line in fp:
            if line.strip() and not line.startswith("#"):
                n, T, l1, l2 = line.split()
                rows[int(n)] = (float(T), float(l1), float(l2))
    return rows


def main():
    rows = golden()
    print("| reading | " + " | ".join(f"{n}^2 L1 / L2" for n in rows) + " |")
    print("|---|" + "---|" * len(rows))
    print("| printed (Table 1) | " + " | ".join(f"{l1:.1e} / {l2:.1e}" for _, l1, l2 in rows.values()) + " |")
    for r in READINGS:
        label, rt, off, nyq, dt, proj = r[:6]
        A = r[6] if len(r) > 6 else 8
        cells = []
        for n, (T, l1p, l2p) in rows.items():
            l1, l2 = O2.test11_errors(n, T, A=A, dt=dt, conserve=proj, R=rt * T, node_offset=off,
                                      zero_nyquist=nyq)
            cells.append(f"{l1:.2e} / {l2:.2e} ({l1 / l1p:.2g}x, {l2 / l2p:.2g}x)")
        print(f"| {label} | " + " | ".join(cells) + " |", flush=True)


if __name__ == "__main__":
    main()
