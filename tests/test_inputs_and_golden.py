"""Synthetic inputs and the paper's bandwidth convention.

* Haar and heat-bath-like generators produce SU(2) links; the heat-bath-like
  ensemble's mean plaquette (measured by the oracle) is the requested 0.6
  (the plaquette of independent links is E[a0]^4).
* Paper Table 1 (Sec. 3): the percent column is per-device bandwidth over the
  MI250X GCD peak of 1.6384 TB/s, and every weak-scaling row has a 48^4
  local volume — the per-GPU share this library benchmarks.
"""
import csv
import os

import numpy as np

from paper_2411_18511_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_bandwidth.csv")


def test_links_are_su2():
    for kind in ("haar", "smeared"):
        U = inputs.gauge_field((4, 2, 2, 4), 1, kind=kind)
        UU = U @ np.conj(np.swapaxes(U, -1, -2))
        assert np.abs(UU - np.eye(2)).max() < 1e-14
        assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_seeded_and_distinct():
    a = inputs.gaussian_spinor((2, 2, 2, 2), 2, 5)
    b = inputs.gaussian_spinor((2, 2, 2, 2), 2, 5)
    c = inputs.gaussian_spinor((2, 2, 2, 2), 2, 6)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    big = inputs.gaussian_spinor((8, 8, 8, 8), 2, 7)
    assert abs(np.mean(np.abs(big) ** 2) - 1.0) < 0.01


def test_smeared_plaquette(oracle):
    eps = inputs.smearing_for_plaquette(0.6)
    assert abs(inputs._mean_a0(eps) ** 4 - 0.6) < 1e-9
    U = inputs.gauge_field((8, 8, 8, 8), 3, kind="smeared")
    assert abs(oracle.plaquette(U) - 0.6) < 0.005
    Uh = inputs.gauge_field((8, 8, 8, 8), 3, kind="haar")
    assert abs(oracle.plaquette(Uh)) < 0.01
    Uu = inputs.gauge_field((4, 4, 4, 4), 0, kind="unit")
    assert oracle.plaquette(Uu) == 1.0


def test_table1_percent_column():
    with open(GOLDEN) as f:
        rows = list(csv.DictReader(line for line in f if not line.startswith("#")))
    assert len(rows) == 13
    for r in rows:
        per_gcd = float(r["tbs"]) / int(r["gcds"])
        assert round(100 * per_gcd / 1.6384) == int(r["pct"])
        vol = int(r["T"]) * int(r["L1"]) * int(r["L2"]) * int(r["L3"])
        if int(r["T"]) != 128:  # weak scaling rows
            assert vol // int(r["gcds"]) == 48 ** 4
