"""Reader of the Table 5.1 fixture (values printed by the paper)."""
from __future__ import annotations

import os

HERE = os.path.dirname(os.path.abspath(__file__))
RESOLUTIONS = (30, 45, 90)
DT = {30: 600.0, 45: 400.0, 90: 200.0}


def load():
    errors, rates = {}, {}
    with open(os.path.join(HERE, "table_5_1_geostrophic.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            f = line.split()
            if f[0] == "rate":
                rates[(f[1], f[2])] = tuple(float(x) for x in f[3:])
            else:
                errors[(f[0], f[1])] = dict(zip(RESOLUTIONS, (float(x) for x in f[2:])))
    return errors, rates
