"""Seeded synthetic inputs for the J-symmetric eigensolver.

This module only draws random numbers and arranges them into the operator
data the solver consumes.  It holds none of the method's arithmetic, so both
the GPU path and the FP64 oracle can take their inputs from it.

Workloads (all Hermitian J-symmetric, J = [[0, -I], [I, 0]]; block form
A = [[A11, A12], [A12^H, A11^T]] with A11^H = A11, A12^T = -A12, Sec. 1,
eq. (blockform)):

* dense:   A11 = (G + G^H)/2, A12 = (H - H^T)/2, G, H i.i.d. complex normal.
* batched: many dense problems of even size n drawn uniformly from 64..1024.
* stencil: a 4D periodic lattice operator with internal dimension d,
  A11 = diag*I - sum_mu (U_mu T_mu + h.c.),
  A12 = scale * sum_mu (B_mu T_mu - (B_mu T_mu)^T),
  with Haar-random unitary links U_mu(x) and complex normal B_mu.
  (T_mu a)(x) = a(x + mu_hat) with periodic wrap.
* known spectrum (Case A, Sec. 4.1): A = U diag(Lambda, Lambda) U^H from a
  J-orthonormal U = [X, J X^*] and Lambda uniform on (0, 1).
* Case B links (Sec. 4.2): Haar-random SU(N) matrices U_mu, mu = 1..4.

Complex normal CN(0,1): real and imaginary parts i.i.d. N(0, 1/2), the real
part drawn first as a whole array.

Vector layout used everywhere: v = [top; bottom], each half of length n/2;
for the stencil each half is site-major (x0 slowest, x3 fastest) with the
internal index fastest.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "cn", "dense_jsym", "batched_sizes", "batched_dense", "haar_unitary",
    "stencil_links", "constant_links", "random_start", "known_spectrum", "haar_su", "STENCIL_DIAG",
    "STENCIL_A12_SCALE",
]

STENCIL_DIAG = 8.1
STENCIL_A12_SCALE = 0.3


def cn(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex normal CN(0,1) array: E|z|^2 = 1."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def dense_jsym(seed_or_rng, h: int):
    """Dense random Hermitian J-symmetric blocks (A11, A12), each h x h complex128."""
    rng = np.random.default_rng(seed_or_rng) if not isinstance(seed_or_rng, np.random.Generator) else seed_or_rng
    G = cn(rng, (h, h))
    H = cn(rng, (h, h))
    A11 = (G + G.conj().T) / 2.0
    A12 = (H - H.T) / 2.0
    return A11, A12


def batched_sizes(seed: int, count: int = 512, nmin: int = 64, nmax: int = 1024):
    """Even sizes drawn uniformly from nmin..nmax (first draw of the batched recipe)."""
    rng = np.random.default_rng(seed)
    n = 2 * rng.integers(nmin // 2, nmax // 2 + 1, count)
    return rng, n.astype(np.int64)


def batched_dense(seed: int, count: int = 512, nmin: int = 64, nmax: int = 1024):
    """List of (A11, A12) for `count` problems of even size in nmin..nmax."""
    rng, n = batched_sizes(seed, count, nmin, nmax)
    probs = []
    for ni in n:
        probs.append(dense_jsym(rng, int(ni) // 2))
    return n, probs


def haar_unitary(rng: np.random.Generator, shape_prefix, d: int) -> np.ndarray:
    """Haar-random d x d unitaries, array of shape shape_prefix + (d, d).

    Gram-Schmidt of the columns of a CN(0,1) matrix, i.e. the QR factor with a
    positive real diagonal of R (Mezzadri, Notices AMS 54, 2007).
    """
    Z = cn(rng, tuple(shape_prefix) + (d, d))
    Q = np.empty_like(Z)
    for c in range(d):
        q = Z[..., :, c].copy()
        for _ in range(2):
            for p in range(c):
                prev = Q[..., :, p]
                proj = np.sum(prev.conj() * q, axis=-1, keepdims=True)
                q = q - prev * proj
        q = q / np.sqrt(np.sum((q.conj() * q).real, axis=-1, keepdims=True))
        Q[..., :, c] = q
    return Q


def _lat(L):
    if np.isscalar(L):
        return (int(L),) * 4
    L = tuple(int(x) for x in L)
    assert len(L) == 4
    return L


def stencil_links(seed: int, L, d: int = 4, b_per_site: bool = False):
    """Random-link stencil data.

    Returns U of shape (4, V, d, d) (Haar per direction and site, site
    lexicographic with x0 slowest) and B of shape (4, d, d) (or (4, V, d, d)
    when b_per_site), complex128.
    """
    L = _lat(L)
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    U = haar_unitary(rng, (4, V), d)
    B = cn(rng, (4, V, d, d) if b_per_site else (4, d, d))
    return U, B


def constant_links(seed: int, L, d: int = 4):
    """Site-independent links: U_mu(x) = U_mu, B_mu constant.

    Returns (U_const (4,d,d), B (4,d,d), U (4,V,d,d) broadcast copy).
    """
    L = _lat(L)
    V = int(np.prod(L))
    rng = np.random.default_rng(seed)
    Uc = haar_unitary(rng, (4,), d)
    B = cn(rng, (4, d, d))
    U = np.ascontiguousarray(np.broadcast_to(Uc[:, None], (4, V, d, d)))
    return Uc, B, U


def haar_su(seed_or_rng, N: int, count: int) -> np.ndarray:
    """count Haar-random SU(N) matrices (count, N, N): the unitary factor of a
    complex Gaussian matrix (QR with a positive real diagonal of R, Mezzadri
    2007), divided by an N-th root of its determinant.  They stand in for the
    Monte Carlo links of the Case B operator (Sec. 4.2)."""
    rng = (seed_or_rng if isinstance(seed_or_rng, np.random.Generator)
           else np.random.default_rng(seed_or_rng))
    out = np.empty((count, N, N), dtype=complex)
    for c in range(count):
        Z = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(2.0)
        Q, R = np.linalg.qr(Z)
        d = np.diag(R)
        Q = Q * (d / np.abs(d))[None, :]
        det = np.linalg.det(Q)
        out[c] = Q / det ** (1.0 / N)
    return out


def random_start(seed: int, n: int) -> np.ndarray:
    """CN(0,1) start vector of length n (not normalised)."""
    return cn(np.random.default_rng(seed), (n,))


def known_spectrum(seed: int, n: int, lam=None):
    """Known-spectrum Hermitian J-symmetric matrix (the Case A recipe, Sec. 4.1).

    A = U diag(Lambda, Lambda) U^H with U = [X, J X^*] (eq. diagblockform),
    Lambda uniform on (0, 1), the entries of X uniform on the square
    (-1, 1) x (-1, 1) i, then made orthonormal column by column against the
    previous columns and their partners J x^* (two Gram-Schmidt passes).
    Returns (A11, A12, Lambda ascending, X)."""
    assert n % 2 == 0
    h = n // 2
    rng = np.random.default_rng(seed)
    if lam is None:
        lam = rng.uniform(0.0, 1.0, h)
    lam = np.asarray(lam, dtype=np.float64)

    def partner(Y):   # J Y^* = [-conj(Y_bot); conj(Y_top)] for the columns of Y
        return np.concatenate([-Y[h:].conj(), Y[:h].conj()], axis=0)

    X = rng.uniform(-1.0, 1.0, (n, h)) + 1j * rng.uniform(-1.0, 1.0, (n, h))
    Q = np.zeros((n, h), dtype=np.complex128)
    Wq = np.zeros((n, h), dtype=np.complex128)   # partners of the columns of Q, kept alongside
    for l in range(h):
        x = X[:, l].copy()
        for _ in range(2):
            if l:
                P = Q[:, :l]
                W = Wq[:, :l]
                x = x - P @ (P.conj().T @ x)
                x = x - W @ (W.conj().T @ x)
        Q[:, l] = x / np.linalg.norm(x)
        Wq[:, l] = partner(Q[:, l:l + 1])[:, 0]
    U = np.concatenate([Q, partner(Q)], axis=1)
    A = (U * np.concatenate([lam, lam])[None, :]) @ U.conj().T
    A = (A + A.conj().T) / 2.0
    A11 = A[:h, :h].copy()
    A12 = A[:h, h:].copy()
    A12 = (A12 - A12.T) / 2.0
    return A11, A12, np.sort(lam), Q
