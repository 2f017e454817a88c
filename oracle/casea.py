"""Known-spectrum Hermitian J-symmetric matrices (the Case A recipe, Sec. 4.1).

Test infrastructure only (see the package docstring).

A = U diag(Lambda, Lambda) U^H with U = [[X1, -X2^*], [X2, X1^*]]
(eq. diagblockform), i.e. U = [X, J X^*] with X = [X1; X2].  Lambda is drawn
uniform on (0, 1); the entries of X uniform on the square
(-1, 1) x (-1, 1) i; then X^H X = I and X^T J X = 0 (equivalently
X1^H X1 + X2^H X2 = I and X1^T X2 - X2^T X1 = 0) are imposed column by column
with a Gram-Schmidt against both the previous columns x_l and their partners
J x_l^*, repeated twice.
"""
from __future__ import annotations

import numpy as np

from .jsym import partner


def known_spectrum(seed: int, n: int, lam=None):
    """Return (A11, A12, Lambda, X).  Lambda (ascending) has n/2 entries; each
    is an exact double eigenvalue of A (to rounding)."""
    assert n % 2 == 0
    h = n // 2
    rng = np.random.default_rng(seed)
    if lam is None:
        lam = rng.uniform(0.0, 1.0, h)
    lam = np.asarray(lam, dtype=np.float64)
    X = rng.uniform(-1.0, 1.0, (n, h)) + 1j * rng.uniform(-1.0, 1.0, (n, h))
    Q = np.zeros((n, h), dtype=np.complex128)
    for l in range(h):
        x = X[:, l].copy()
        for _ in range(2):
            if l:
                P = Q[:, :l]
                W = partner(P)
                x = x - P @ (P.conj().T @ x)
                x = x - W @ (W.conj().T @ x)
        Q[:, l] = x / np.linalg.norm(x)
    U = np.concatenate([Q, partner(Q)], axis=1)
    A = (U * np.concatenate([lam, lam])[None, :]) @ U.conj().T
    A = (A + A.conj().T) / 2.0
    A11 = A[:h, :h].copy()
    A12 = A[:h, h:].copy()
    A12 = (A12 - A12.T) / 2.0
    return A11, A12, np.sort(lam), Q
