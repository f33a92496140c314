"""Independent dense assembly of the HEOM generator, for pinning the oracle.

The hierarchy is enumerated here by brute force (itertools over all tuples with
entries 0..D, kept if the sum is <= D), and every superoperator is built from
its operator definition with Kronecker products instead of the element masks
the oracle uses:

    V^x A = V A - A V,   V^o A = V A + A V,   V^x V^x = (V^x)^2,
    -i [H, A] = -i (H A - A H),

with row-major vectorisation vec(A X B) = (A kron B^T) vec(X).  Bath weights
come from the oracle's coefficient routine, which is pinned separately against
quadrature of the spectral density.  The ADO order (level, then descending
lexicographic tuple) is the same convention the oracle documents.
"""

from __future__ import annotations

import itertools

import numpy as np

TWO_PI_C = 2.0 * np.pi * 2.99792458e-5


def enumerate_tuples(W, D):
    tups = [t for t in itertools.product(range(D + 1), repeat=W) if sum(t) <= D]
    tups.sort(key=lambda t: (sum(t), tuple(-x for x in t)))
    return tups


def modes_of(prob, orc):
    """[(site, k, gamma, c, lamnu)] bath-major, plus per-bath (site, Delta)."""
    modes, baths = [], []
    for b in prob["baths"]:
        g, c, lamnu, delta = orc.bath_coefficients(b["lambda_cm"], b["tau_fs"],
                                                   prob["temperature_K"], b["matsubara"])
        for k in range(b["matsubara"] + 1):
            modes.append((b["state"], k, g[k], c[k], lamnu if k == 0 else 0.0))
        baths.append((b["state"], delta))
    return modes, baths


def liouvillian(prob, orc, rescale=True, terminator=True, gauge=1.0, add_reorg=False):
    H = np.array(prob["H"], dtype=np.complex128)
    if add_reorg:
        # eq. h-ex: the site energy carries the reorganisation energy of its bath
        for b in prob["baths"]:
            H[b["state"], b["state"]] += b["lambda_cm"]
    H = H * TWO_PI_C
    N = H.shape[0]
    D = prob["depth"]
    modes, baths = modes_of(prob, orc)
    W = len(modes)
    tups = enumerate_tuples(W, D)
    index = {t: u for u, t in enumerate(tups)}
    I = np.eye(N)
    NN = N * N

    def left(A):
        return np.kron(A, I)

    def right(A):
        return np.kron(I, A.T)

    def proj(s):
        V = np.zeros((N, N))
        V[s, s] = 1.0
        return V

    comm = -1j * (left(H) - right(H))
    L = np.zeros((len(tups) * NN, len(tups) * NN), dtype=np.complex128)
    for u, t in enumerate(tups):
        blk = slice(u * NN, (u + 1) * NN)
        damp = sum(t[l] * modes[l][2] for l in range(W))
        diag = comm - damp * np.eye(NN)
        if terminator:
            for s, delta in baths:
                Vx = left(proj(s)) - right(proj(s))
                diag = diag - delta * (Vx @ Vx)
        L[blk, blk] += diag
        for l, (s, k, g, c, lamnu) in enumerate(modes):
            V = proj(s)
            Vx = left(V) - right(V)
            Vo = left(V) + right(V)
            ac = abs(c) if abs(c) > 0 else 1.0
            if sum(t) < D:
                tp = list(t)
                tp[l] += 1
                v = index[tuple(tp)]
                a = np.sqrt((t[l] + 1) * ac) if rescale else 1.0
                L[blk, v * NN:(v + 1) * NN] += gauge * 1j * a * Vx
            if t[l] > 0:
                tm = list(t)
                tm[l] -= 1
                v = index[tuple(tm)]
                a = np.sqrt(t[l] / ac) if rescale else float(t[l])
                theta = 1j * c * Vx + (lamnu * Vo if k == 0 else 0.0)
                L[blk, v * NN:(v + 1) * NN] += gauge * a * theta
    return L, tups


def rk4_matrix(L, h):
    """One classic RK4 step of dy/dt = L y as a matrix polynomial."""
    hL = h * L
    I = np.eye(L.shape[0])
    hL2 = hL @ hL
    hL3 = hL2 @ hL
    return I + hL + hL2 / 2.0 + hL3 / 6.0 + hL3 @ hL / 24.0
