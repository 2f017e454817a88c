"""Pins for the Case B operator of the oracle (Sec. 4.2 and the appendix):
the printed gamma matrices and their algebra, the su(N) basis, the adjoint
representation, eqs. G5Hermit and MayoranaProp, the J-symmetry of A = D D^H
with J = C gamma_5, the matrix-free form against the dense definition, and
the canonical reordering of J.  CPU only."""
import numpy as np
import pytest

from oracle import jsym, tek, trlan

KAPPA = 0.12


def _us(seed, N):
    return tek.haar_su(np.random.default_rng(seed), N, 4)


def test_gamma_algebra_as_printed():
    G = tek.GAMMA + [tek.G5]
    for m in range(5):
        assert np.allclose(G[m], G[m].conj().T)
        for v in range(5):
            assert np.allclose(G[m] @ G[v] + G[v] @ G[m], 2.0 * (m == v) * np.eye(4))
    # gamma_5 = gamma_4 gamma_1 gamma_2 gamma_3 is the printed real matrix
    printed = np.array([[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]])
    assert np.array_equal(tek.G5, printed)
    # transposes: gamma_1, gamma_3 antisymmetric; gamma_2, gamma_4, gamma_5 symmetric
    for m, sign in zip(range(5), (-1, 1, -1, 1, 1)):
        assert np.allclose(G[m].T, sign * G[m])


def test_charge_conjugation_and_J():
    C = tek.C
    assert np.allclose(np.linalg.inv(C), -C) and np.allclose(np.linalg.inv(C), C.T)
    for g in tek.GAMMA:
        assert np.allclose(C @ g @ C.T, -g.T)          # eq. (CCGamma)
    J = tek.J4
    assert np.allclose(J.imag, 0)
    J = J.real
    assert np.allclose(J.T, -J) and np.allclose(J @ J, -np.eye(4))
    assert np.allclose(C @ tek.G5, tek.G5 @ C)


@pytest.mark.parametrize("N", [2, 3, 5])
def test_su_generators(N):
    T = tek.su_generators(N)
    assert T.shape == (N * N - 1, N, N)
    G = np.einsum("aij,bji->ab", T, T)
    assert np.allclose(G, 0.5 * np.eye(N * N - 1))
    assert np.allclose(T, np.conj(np.transpose(T, (0, 2, 1))))
    assert np.allclose(np.einsum("aii->a", T), 0)


def test_haar_su_and_adjoint_representation():
    N = 4
    U = _us(1, N)
    T = tek.su_generators(N)
    for u in U:
        assert np.allclose(u @ u.conj().T, np.eye(N)) and np.isclose(np.linalg.det(u), 1.0)
    V0, V1 = tek.adjoint(U[0], T), tek.adjoint(U[1], T)
    assert np.allclose(V0 @ V0.T, np.eye(N * N - 1))
    # a group homomorphism: Ad(U0 U1) = Ad(U0) Ad(U1)
    assert np.allclose(tek.adjoint(U[0] @ U[1], T), V0 @ V1)
    # and Ad(U^H) = Ad(U)^T
    assert np.allclose(tek.adjoint(U[0].conj().T, T), V0.T)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_matrix_free_matches_dense(N):
    Us = _us(2, N)
    D = tek.dense_D(Us, KAPPA)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(D.shape[0]) + 1j * rng.standard_normal(D.shape[0])
    assert np.allclose(tek.apply_D(Us, KAPPA, psi), D @ psi)
    assert np.allclose(tek.apply_D(Us, KAPPA, psi, dagger=True), D.conj().T @ psi)
    assert np.allclose(tek.apply_A(Us, KAPPA, psi), D @ (D.conj().T @ psi))


def test_eq_g5hermit_mayorana_and_J_symmetry():
    N = 3
    Us = _us(4, N)
    na = N * N - 1
    D = tek.dense_D(Us, KAPPA)
    G5 = np.kron(tek.G5, np.eye(na))
    Cf = np.kron(tek.C, np.eye(na))
    assert np.allclose(G5 @ D @ G5, D.conj().T)          # eq. (G5Hermit)
    assert np.allclose(Cf @ D @ Cf.T, D.T)               # eq. (MayoranaProp)
    A = tek.dense_A(Us, KAPPA)
    assert np.allclose(A, A.conj().T)
    assert np.allclose(A, (D @ G5) @ (D @ G5))           # A = (D gamma_5)^2
    Jf = np.kron(tek.J4.real, np.eye(na))
    assert np.allclose(Jf @ A @ np.linalg.inv(Jf), A.T)  # J-symmetric
    w = np.linalg.eigvalsh(A)
    assert w[0] > -1e-12
    assert np.abs(w[0::2] - w[1::2]).max() < 1e-10 * w[-1]   # doubly degenerate


def test_canonical_pairing_gives_block_form():
    N = 3
    Us = _us(5, N)
    na = N * N - 1
    A = tek.dense_A(Us, KAPPA)
    Jf = np.kron(tek.J4.real, np.eye(na))
    P = tek.canonical_matrix(Jf)
    n = 4 * na
    assert np.allclose(P.T @ P, np.eye(n))
    assert np.allclose(P.T @ Jf @ P, jsym.J_matrix(n))
    Ac = P.T @ A @ P
    h = n // 2
    A11, A12 = Ac[:h, :h], Ac[:h, h:]
    assert np.allclose(Ac, jsym.dense_from_blocks(A11, A12))
    assert np.allclose(A12.T, -A12) and np.allclose(A11, A11.conj().T)
    # this J pairs spins (0, 1) and (2, 3) with sign +1: top = spins 0, 2
    top, bot, sgn = tek.canonical_pairing(tek.J4.real)
    assert list(top) == [0, 2] and list(bot) == [1, 3] and (sgn == 1).all()


def test_trlan_on_canonical_tek_vs_brute():
    N = 4
    Us = _us(6, N)
    na = N * N - 1
    A = tek.dense_A(Us, KAPPA)
    P = tek.canonical_matrix(np.kron(tek.J4.real, np.eye(na)))
    Ac = P.T @ A @ P
    ref, _ = jsym.brute(Ac)
    out = trlan.trlan_jsym(lambda v: Ac @ v, Ac.shape[0], 6, 12, 28, 1e-10)
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - ref[:6]).max() < 1e-10 * ref[-1]


@pytest.mark.parametrize("N", [2, 3, 6])
def test_entry_formulas_match_generator_sums(N):
    rng = np.random.default_rng(N)
    na = N * N - 1
    psi = rng.standard_normal((3, na)) + 1j * rng.standard_normal((3, na))
    X = tek.coef_to_mat(psi, N)
    assert np.allclose(tek.coef_to_mat_entries(psi, N), X)
    Y = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    Y -= np.trace(Y, axis1=1, axis2=2)[:, None, None] * np.eye(N) / N     # traceless
    assert np.allclose(tek.mat_to_coef_entries(Y, N), tek.mat_to_coef(Y, N))
    Us = _us(7, N)
    v = rng.standard_normal(4 * na) + 1j * rng.standard_normal(4 * na)
    assert np.allclose(tek.apply_A(Us, KAPPA, v, entries=True), tek.apply_A(Us, KAPPA, v))


def test_canonical_layout_helpers():
    N = 3
    na = N * N - 1
    Jf = np.kron(tek.J4.real, np.eye(na))
    P = tek.canonical_matrix(Jf)
    v = np.arange(4 * na) + 0j
    assert np.allclose(tek.from_canonical(v, na), P @ v)
    assert np.allclose(tek.to_canonical(P @ v, na), v)
