"""J-structure, operators and brute-force spectra (FP64, plain NumPy).

Test infrastructure only (see the package docstring).

Notation follows Sec. 1 of the paper: J = [[0, -I], [I, 0]] (real, J^T = -J =
J^-1), a Hermitian J-symmetric A satisfies J A J^-1 = A^T (eq. symmetry) and has
the block form A = [[A11, A12], [A12^H, A11^T]] with A11^H = A11 and
A12^T = -A12 (eq. blockform).  Each eigenvalue is doubly degenerate with
partner eigenvector y = J x^* (eq. pairev).
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# J and partners (Sec. 1, eqs. symmetry and pairev)
# --------------------------------------------------------------------------
def J_matrix(n: int) -> np.ndarray:
    """The canonical J = [[0, -I], [I, 0]] as a dense real n x n matrix."""
    assert n % 2 == 0
    h = n // 2
    J = np.zeros((n, n))
    J[:h, h:] = -np.eye(h)
    J[h:, :h] = np.eye(h)
    return J


def J_apply(x: np.ndarray) -> np.ndarray:
    """J x for x of shape (n,) or (n, k): [a; b] -> [-b; a]."""
    h = x.shape[0] // 2
    return np.concatenate([-x[h:], x[:h]], axis=0)


def partner(x: np.ndarray) -> np.ndarray:
    """Partner eigenvector y = J x^* (eq. pairev); columnwise for 2D input."""
    return J_apply(np.conj(x))


# --------------------------------------------------------------------------
# Dense block form (eq. blockform)
# --------------------------------------------------------------------------
def dense_from_blocks(A11: np.ndarray, A12: np.ndarray) -> np.ndarray:
    """A = [[A11, A12], [A12^H, A11^T]]."""
    return np.block([[A11, A12], [A12.conj().T, A11.T]])


# --------------------------------------------------------------------------
# 4D periodic J-stencil.  Sites are lexicographic with x0 slowest; a half
# vector is (L0, L1, L2, L3, d).  (T_mu a)(x) = a(x + mu_hat).
#   A11 = diag*I - sum_mu (U_mu T_mu + (U_mu T_mu)^H)
#   A12 = scale * sum_mu (B_mu T_mu - (B_mu T_mu)^T)
# --------------------------------------------------------------------------
def _lat(L):
    if np.isscalar(L):
        return (int(L),) * 4
    return tuple(int(x) for x in L)


def _site_links(M, mu, L, d):
    """Link field of direction mu as (L0,L1,L2,L3,d,d) (broadcast if constant)."""
    if M.ndim == 3:                       # site independent: (4, d, d)
        return M[mu].reshape((1, 1, 1, 1, d, d))
    return M[mu].reshape(tuple(L) + (d, d))


def _mv(M, a):        # M(x) a(x)
    return np.einsum("...ij,...j->...i", M, a)


def _mhv(M, a):       # M(x)^H a(x)
    return np.einsum("...ji,...j->...i", M.conj(), a)


def _mtv(M, a):       # M(x)^T a(x)
    return np.einsum("...ji,...j->...i", M, a)


def _mcv(M, a):       # conj(M(x)) a(x)
    return np.einsum("...ij,...j->...i", M.conj(), a)


def _fwd(a, mu):      # a(x + mu_hat)
    return np.roll(a, -1, axis=mu)


def _bwd(a, mu):      # a(x - mu_hat)
    return np.roll(a, 1, axis=mu)


def stencil_apply(U, B, L, v, diag=8.1, scale=0.3):
    """y = A v for the 4D J-stencil, directly from the operator definitions.

    U: (4, V, d, d); B: (4, d, d) or (4, V, d, d).  v: (n,) complex, n = 2*V*d.
    The bottom half uses the explicit transposes/adjoints of the hopping terms
    (A12^H and A11^T written out, not derived from the symmetry).
    """
    L = _lat(L)
    d = U.shape[-1]
    V = int(np.prod(L))
    h = V * d
    a = v[:h].reshape(L + (d,))
    b = v[h:].reshape(L + (d,))
    top = diag * a + 0j
    bot = diag * b + 0j
    for mu in range(4):
        Um = _site_links(U, mu, L, d)
        Bm = _site_links(B, mu, L, d)
        # A11 a = diag a - sum_mu [U(x) a(x+mu) + U(x-mu)^H a(x-mu)]
        top -= _mv(Um, _fwd(a, mu)) + _bwd(_mhv(Um, a), mu)
        # A12 b = scale sum_mu [B(x) b(x+mu) - B(x-mu)^T b(x-mu)]
        top += scale * (_mv(Bm, _fwd(b, mu)) - _bwd(_mtv(Bm, b), mu))
        # A12^H a = scale sum_mu [B(x-mu)^H a(x-mu) - conj(B(x)) a(x+mu)]
        bot += scale * (_bwd(_mhv(Bm, a), mu) - _mcv(Bm, _fwd(a, mu)))
        # A11^T b = diag b - sum_mu [U(x-mu)^T b(x-mu) + conj(U(x)) b(x+mu)]
        bot -= _bwd(_mtv(Um, b), mu) + _mcv(Um, _fwd(b, mu))
    return np.concatenate([top.reshape(-1), bot.reshape(-1)])


def stencil_blocks_dense(U, B, L, diag=8.1, scale=0.3):
    """Materialise A11 and A12 of the stencil as dense (V*d)^2 matrices by an
    explicit loop over sites and directions (small lattices only)."""
    L = _lat(L)
    d = U.shape[-1]
    V = int(np.prod(L))
    strides = (L[1] * L[2] * L[3], L[2] * L[3], L[3], 1)

    def site(x):
        return sum(int(x[i]) * strides[i] for i in range(4))

    def coords(s):
        c = []
        for i in range(4):
            c.append(s // strides[i])
            s %= strides[i]
        return c

    def link(M, mu, s):
        return M[mu] if M.ndim == 3 else M[mu, s]

    A11 = np.zeros((V * d, V * d), dtype=np.complex128)
    A12 = np.zeros((V * d, V * d), dtype=np.complex128)
    for s in range(V):
        x = coords(s)
        A11[s * d:(s + 1) * d, s * d:(s + 1) * d] += diag * np.eye(d)
        for mu in range(4):
            xf = list(x); xf[mu] = (xf[mu] + 1) % L[mu]
            xb = list(x); xb[mu] = (xb[mu] - 1) % L[mu]
            sf, sb = site(xf), site(xb)
            A11[s * d:(s + 1) * d, sf * d:(sf + 1) * d] -= link(U, mu, s)
            A11[s * d:(s + 1) * d, sb * d:(sb + 1) * d] -= link(U, mu, sb).conj().T
            A12[s * d:(s + 1) * d, sf * d:(sf + 1) * d] += scale * link(B, mu, s)
            A12[s * d:(s + 1) * d, sb * d:(sb + 1) * d] -= scale * link(B, mu, sb).T
    return A11, A12


def stencil_dense(U, B, L, diag=8.1, scale=0.3):
    """Dense A of the stencil (small lattices only)."""
    A11, A12 = stencil_blocks_dense(U, B, L, diag, scale)
    return dense_from_blocks(A11, A12)


def constant_link_spectrum(Uc, B, L, diag=8.1, scale=0.3):
    """All n eigenvalues (ascending) of the stencil with site-independent links.

    With U_mu(x) = U_mu and constant B_mu the operator is diagonal in momentum:
    a(x) = alpha e^{i k.x}, b(x) = beta e^{i k.x}, k_mu = 2 pi n_mu / L_mu, and
    (alpha, beta) -> M(k) (alpha, beta) with the 2d x 2d Hermitian block
      M(k) = [[F(k), G(k)], [-conj(G(-k)), conj(F(-k))]],
      F(k) = diag I - sum_mu (U_mu e^{i k_mu} + U_mu^H e^{-i k_mu}),
      G(k) = scale sum_mu (B_mu e^{i k_mu} - B_mu^T e^{-i k_mu}).
    The spectrum of A is the union over k of eig(M(k)).
    """
    L = _lat(L)
    d = Uc.shape[-1]
    ks = [2 * np.pi * np.arange(Lm) / Lm for Lm in L]
    K = np.stack(np.meshgrid(*ks, indexing="ij"), axis=-1).reshape(-1, 4)  # (V, 4)

    def F(Kv):
        out = np.broadcast_to(diag * np.eye(d), (Kv.shape[0], d, d)).astype(np.complex128)
        for mu in range(4):
            ph = np.exp(1j * Kv[:, mu])[:, None, None]
            out = out - (Uc[mu][None] * ph + Uc[mu].conj().T[None] * ph.conj())
        return out

    def G(Kv):
        out = np.zeros((Kv.shape[0], d, d), dtype=np.complex128)
        for mu in range(4):
            ph = np.exp(1j * Kv[:, mu])[:, None, None]
            out = out + scale * (B[mu][None] * ph - B[mu].T[None] * ph.conj())
        return out

    evs = []
    chunk = 1 << 16
    for s in range(0, K.shape[0], chunk):
        Kc = K[s:s + chunk]
        M = np.empty((Kc.shape[0], 2 * d, 2 * d), dtype=np.complex128)
        M[:, :d, :d] = F(Kc)
        M[:, :d, d:] = G(Kc)
        M[:, d:, :d] = -G(-Kc).conj()
        M[:, d:, d:] = F(-Kc).conj()
        evs.append(np.linalg.eigvalsh(M).reshape(-1))
    return np.sort(np.concatenate(evs))


# --------------------------------------------------------------------------
# Brute force (dense eigh)
# --------------------------------------------------------------------------
def pair_eigenvalues(all_ev: np.ndarray, which: str = "lowest"):
    """Distinct J-pair eigenvalues from the full ascending spectrum: every
    eigenvalue appears twice (Sec. 1), so take every second one.  Returns the
    pair values in the requested order and the largest gap inside a pair."""
    ev = np.sort(all_ev)
    gaps = np.abs(ev[1::2] - ev[0::2])
    pairs = ev[0::2]
    if which == "largest":
        pairs = ev[1::2][::-1]
    return pairs, float(gaps.max()) if gaps.size else 0.0


def brute(A: np.ndarray, which: str = "lowest"):
    """All distinct pair eigenvalues of a dense Hermitian J-symmetric A by
    numpy.linalg.eigvalsh; also returns the largest in-pair gap."""
    return pair_eigenvalues(np.linalg.eigvalsh(A), which)
