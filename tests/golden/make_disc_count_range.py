"""Write disc_count_range_nside128.txt: min/max disc sizes over all NSIDE-128 pixel-centre pointings.

Calls only the oracle (pixel centres from its pix2ang, counts from its
plain all-candidate-pixel disc scan).  Run from the repository root:
    python tests/golden/make_disc_count_range.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

NSIDE = 128
RADII = (5.0, 7.5, 10.0, 15.0, 20.0, 25.0, 30.0)


def main():
    pix = np.arange(12 * NSIDE * NSIDE)
    th, ph = oracle.pix2ang(NSIDE, pix)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "disc_count_range_nside128.txt")
    lines = ["# Disc sizes (pixel centres within rho, inclusive) over every NSIDE-128",
             "# pixel-centre pointing, from the oracle's disc scan (make_disc_count_range.py).",
             "# columns: rho_max_deg  min_count  argmin_pix  max_count  argmax_pix"]
    for r in RADII:
        c = oracle.disc_counts(NSIDE, th, ph, np.deg2rad(r))
        lines.append(f"{r:5.1f} {c.min():6d} {int(c.argmin()):6d} {c.max():6d} {int(c.argmax()):6d}")
        print(lines[-1], flush=True)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
