"""Writes the stored expected values of tests/golden from closed forms and oracle/ only."""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tcinputs as T  # noqa: E402
from oracle.heg import gb_delta  # noqa: E402

w = T.workload("heg14_g16")
L = float(w.lattice[0, 0])
d = gb_delta(w.lattice, w.kmesh, w.alpha)
out = {
    "source": "closed-form lattice sum over the 7 occupied plane waves; Eq. correction2 / divcorr_2ax_scf",
    "L_bohr": L,
    "alpha": w.alpha,
    "exchange_uncorrected_Ha": -25.5 / (math.pi * L),
    "four_pi_dgb_over_omega": 4 * math.pi * d / w.omega,
    "exchange_corrected_Ha": -25.5 / (math.pi * L) - 2 * 7 * (4 * math.pi * d / w.omega) / 2,
    "madelung_sc_over_L": 2.837297 / L,
}
with open(os.path.join(HERE, "heg_hf_exchange.json"), "w") as fh:
    json.dump(out, fh, indent=1)
print(out)
