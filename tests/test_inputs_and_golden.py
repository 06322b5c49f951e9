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


def _abelian_flux(dims, mu, nu, n):
    """Diagonal SU(2) links diag(e^{i a}, e^{-i a}) with a = phi x_mu on the
    nu-links and 1 elsewhere, phi = 2 pi n / L_mu: every (mu, nu) plaquette
    carries the phase phi (also across the periodic boundary, where the jump of
    a is -phi (L_mu - 1) = phi mod 2 pi), every other plaquette is 1."""
    phi = 2 * np.pi * n / dims[mu]
    U = np.zeros((4,) + tuple(dims) + (2, 2), dtype=np.complex128)
    U[..., 0, 0] = 1
    U[..., 1, 1] = 1
    x = np.indices(dims)[mu]
    U[nu, ..., 0, 0] = np.exp(1j * phi * x)
    U[nu, ..., 1, 1] = np.exp(-1j * phi * x)
    return U, phi


def test_plaquette_constant_flux_closed_form(oracle):
    """Mean plaquette (1/2) Re tr over the six planes: one plane at cos(phi),
    five at 1, so (5 + cos phi) / 6 -- for each plane and either orientation of
    the flux, which a misplaced dagger or a wrong neighbour site would change
    (the phase would cancel or double)."""
    dims = (4, 6, 8, 4)
    for mu, nu in ((1, 2), (0, 3), (2, 0), (3, 1)):
        for n in (1, 2):
            U, phi = _abelian_flux(dims, mu, nu, n)
            assert abs(oracle.plaquette(U) - (5 + np.cos(phi)) / 6) < 1e-14, (mu, nu, n)


def test_plaquette_gauge_invariance(oracle):
    """P[U^g] = P[U] with U^g_mu(x) = g(x) U_mu(x) g(x + mu)^+ for random SU(2)
    g, on Haar links (any wrong orientation or site of a link in the loop
    leaves g factors that do not cancel)."""
    dims = (4, 2, 6, 4)
    U = inputs.gauge_field(dims, 11, kind="haar")
    g = inputs.gauge_field(dims, 12, kind="haar")[0]  # one SU(2) matrix per site
    Ug = np.empty_like(U)
    for mu in range(4):
        gs = np.roll(g, -1, axis=mu)  # g(x + mu)
        Ug[mu] = g @ U[mu] @ np.conj(np.swapaxes(gs, -1, -2))
    p0, p1 = oracle.plaquette(U), oracle.plaquette(Ug)
    assert abs(p0 - p1) < 1e-14
    assert abs(p0) > 1e-3  # a nontrivial value, not a cancellation to 0
