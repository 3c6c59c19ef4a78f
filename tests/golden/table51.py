"""Reader of the Table 5.1 fixture (values printed by the paper)."""
from __future__ import annotations

import os

HERE = os.path.dirname(os.path.abspath(__file__))
RESOLUTIONS = (30, 45, 90, 180, 360)
# time steps of section 5.1 at each resolution (s)
DT = {30: 600.0, 45: 400.0, 90: 200.0, 180: 100.0, 360: 50.0}


def load():
    """errors[(scheme, norm)][n] and rates[(scheme, norm)][n] (the rate from
    the previous resolution to n); None where the table prints nothing."""
    errors, rates = {}, {}
    with open(os.path.join(HERE, "table_5_1_geostrophic.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            f = line.split()
            vals = [None if x == "-" else float(x) for x in f[-len(RESOLUTIONS):]]
            if f[0] == "rate":
                rates[(f[1], f[2])] = dict(zip(RESOLUTIONS, vals))
            else:
                errors[(f[0], f[1])] = dict(zip(RESOLUTIONS, vals))
    return errors, rates
