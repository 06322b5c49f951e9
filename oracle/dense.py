"""Dense-matrix Wilson-Dirac builder for tiny lattices — TEST INFRASTRUCTURE ONLY.

A second, independent construction of D as an explicit matrix, assembled
block by block from Kronecker products (spin matrix) x (colour matrix).  It
shares no code with ``oracle.c`` (it builds its own gamma matrices from the
Pauli matrices) and is used to pin the oracle by brute force: spectra,
determinants, Schur complements and dense solves on 2^4 .. 4^4 lattices.

Row/column index of (site, spin a, colour i) is (lex * 4 + a) * N + i with
lex = ((t*L1 + x1)*L2 + x2)*L3 + x3, matching the natural field layout.
"""
import itertools

import numpy as np

PAULI = [
    np.array([[0, 1], [1, 0]], np.complex128),
    np.array([[0, -1j], [1j, 0]], np.complex128),
    np.array([[1, 0], [0, -1]], np.complex128),
]


def gammas():
    """Chiral-basis gamma matrices built from 2x2 blocks."""
    z = np.zeros((2, 2), np.complex128)
    one = np.eye(2, dtype=np.complex128)
    out = [np.block([[z, one], [one, z]])]
    for s in PAULI:
        out.append(np.block([[z, -1j * s], [1j * s, z]]))
    return out


def _sites(dims):
    return list(itertools.product(*[range(n) for n in dims]))


def _lex(dims, x):
    return ((x[0] * dims[1] + x[1]) * dims[2] + x[2]) * dims[3] + x[3]


def dirac_matrix(U, m0):
    """Dense D for gauge field U of shape [4, T, L1, L2, L3, N, N]."""
    dims = U.shape[1:5]
    n = U.shape[-1]
    V = int(np.prod(dims))
    blk = 4 * n
    D = np.zeros((V * blk, V * blk), np.complex128)
    G = gammas()
    one4 = np.eye(4, dtype=np.complex128)
    for x in _sites(dims):
        s = _lex(dims, x)
        D[s * blk:(s + 1) * blk, s * blk:(s + 1) * blk] += (4.0 + m0) * np.eye(blk)
        for mu in range(4):
            # forward neighbour x + mu, hop sign -1 when leaving t = T-1
            y = list(x)
            y[mu] = (x[mu] + 1) % dims[mu]
            sf = _lex(dims, y)
            sign_f = -1.0 if (mu == 0 and x[0] == dims[0] - 1) else 1.0
            blockf = np.kron(one4 - G[mu], U[mu][tuple(x)])
            D[s * blk:(s + 1) * blk, sf * blk:(sf + 1) * blk] += -0.5 * sign_f * blockf
            # backward neighbour x - mu, hop sign of the link (x - mu, mu)
            y = list(x)
            y[mu] = (x[mu] - 1) % dims[mu]
            sb = _lex(dims, y)
            sign_b = -1.0 if (mu == 0 and y[0] == dims[0] - 1) else 1.0
            blockb = np.kron(one4 + G[mu], U[mu][tuple(y)].conj().T)
            D[s * blk:(s + 1) * blk, sb * blk:(sb + 1) * blk] += -0.5 * sign_b * blockb
    return D


def parity_index(dims, n):
    """Row indices of the even and of the odd sites (each with its 4N components)."""
    blk = 4 * n
    ev, od = [], []
    for x in _sites(dims):
        s = _lex(dims, x)
        rows = list(range(s * blk, (s + 1) * blk))
        (ev if sum(x) % 2 == 0 else od).extend(rows)
    return np.array(ev), np.array(od)


def schur_blocks(D, dims, n):
    """(D_ee, D_eo, D_oe, D_oo) blocks of a dense D."""
    e, o = parity_index(dims, n)
    return D[np.ix_(e, e)], D[np.ix_(e, o)], D[np.ix_(o, e)], D[np.ix_(o, o)]


def free_spectrum(dims, m0, n):
    """Closed-form eigenvalues of the free (U = 1) operator.

    With p_k = 2 pi n_k / L_k (periodic) and p_0 = (2 pi n_0 + pi) / T
    (antiperiodic), lambda = m0 + sum(1 - cos p) +- i sqrt(sum sin^2 p), each
    sign with multiplicity 2N.
    """
    ev = []
    for nn in itertools.product(*[range(L) for L in dims]):
        p = [(2 * np.pi * nn[0] + np.pi) / dims[0]] + [2 * np.pi * nn[k] / dims[k] for k in (1, 2, 3)]
        re = m0 + sum(1 - np.cos(q) for q in p)
        im = np.sqrt(sum(np.sin(q) ** 2 for q in p))
        ev += [re + 1j * im] * (2 * n) + [re - 1j * im] * (2 * n)
    return np.array(ev)
