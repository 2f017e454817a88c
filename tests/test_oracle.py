"""Pins for the FP64 oracle: each check ties it to something other than itself
(the paper's invariants, brute-force diagonalisation, closed forms, values the
paper prints).  CPU only."""
import json
import math
import os

import numpy as np
import pytest

from paper_2001_07428_amd import inputs
from oracle import jsym, trlan

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(seed, h):
    A11, A12 = inputs.dense_jsym(seed, h)
    return jsym.dense_from_blocks(A11, A12)


# ---------------------------------------------------------------- structure
def test_dense_generator_is_hermitian_jsymmetric():
    A = _dense(1, 100)
    J = jsym.J_matrix(200)
    assert np.abs(A - A.conj().T).max() == 0.0
    # J A J^-1 = A^T with J^-1 = J^T (Sec. 1, eq. symmetry)
    assert np.abs(J @ A @ J.T - A.T).max() == 0.0
    assert np.allclose(J.T, -J) and np.allclose(J.T @ J, np.eye(200))


def test_J_apply_and_partner_match_matrix():
    rng = np.random.default_rng(0)
    x = inputs.cn(rng, (12, 3))
    J = jsym.J_matrix(12)
    assert np.allclose(jsym.J_apply(x), J @ x, atol=0, rtol=0)
    assert np.allclose(jsym.partner(x), J @ x.conj(), atol=0, rtol=0)


def test_lemma1_w_orthogonal_and_A_orthogonal():
    """Lemma 1: w = J v^* satisfies w^H v = 0 and w^H A v = 0 for any v."""
    A = _dense(3, 60)
    rng = np.random.default_rng(1)
    for _ in range(5):
        v = inputs.cn(rng, 120)
        w = jsym.partner(v)
        assert abs(np.vdot(w, v)) < 1e-13 * np.linalg.norm(v) ** 2
        assert abs(np.vdot(w, A @ v)) < 1e-12 * np.linalg.norm(v) ** 2 * np.linalg.norm(A, 2)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (3, 3, 3, 3), (2, 3, 2, 3)])
@pytest.mark.parametrize("b_per_site", [False, True])
def test_stencil_apply_matches_site_loop(L, b_per_site):
    """Two independent codings of the stencil definition agree (roll-based
    apply vs explicit site/direction loop); L=2 has x+mu == x-mu."""
    U, B = inputs.stencil_links(4, L, b_per_site=b_per_site)
    Ad = jsym.stencil_dense(U, B, L)
    n = Ad.shape[0]
    J = jsym.J_matrix(n)
    assert np.abs(Ad - Ad.conj().T).max() == 0.0
    assert np.abs(J @ Ad @ J.T - Ad.T).max() < 1e-15
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = inputs.cn(rng, n)
        assert np.abs(jsym.stencil_apply(U, B, L, v) - Ad @ v).max() < 1e-13


@pytest.mark.parametrize("L", [(3, 3, 3, 3), (2, 3, 4, 3)])
def test_constant_link_closed_form(L):
    """Fourier block diagonalisation of the constant-link stencil reproduces
    the dense spectrum (independent of both stencil codings)."""
    Uc, B, U = inputs.constant_links(6, L)
    Ad = jsym.stencil_dense(U, B, L)
    ev = np.linalg.eigvalsh(Ad)
    cf = jsym.constant_link_spectrum(Uc, B, L)
    assert np.abs(ev - cf).max() < 1e-12


def test_haar_links_unitary():
    U, _ = inputs.stencil_links(4, (2, 2, 2, 2))
    I = np.eye(4)
    assert np.abs(np.einsum("...ji,...jk->...ik", U.conj(), U) - I).max() < 1e-14


@pytest.mark.parametrize("case", ["dense", "stencil", "casea"])
def test_exact_double_degeneracy(case):
    """Every eigenvalue of a Hermitian J-symmetric matrix is doubly degenerate."""
    if case == "dense":
        A = _dense(1, 100)
    elif case == "stencil":
        U, B = inputs.stencil_links(4, 3)
        A = jsym.stencil_dense(U, B, 3)
    else:
        A11, A12, _, _ = inputs.known_spectrum(8, 200)
        A = jsym.dense_from_blocks(A11, A12)
    _, gap = jsym.brute(A)
    assert gap < 1e-12 * np.linalg.norm(A, 2)


def test_known_spectrum_generator():
    """Case A recipe: A = [X, JX*] diag(L, L) [X, JX*]^H with the constraints
    X1^H X1 + X2^H X2 = I and X1^T X2 - X2^T X1 = 0 (eq. diagblockform)."""
    n = 160
    A11, A12, lam, Q = inputs.known_spectrum(8, n)
    h = n // 2
    X1, X2 = Q[:h], Q[h:]
    assert np.abs(X1.conj().T @ X1 + X2.conj().T @ X2 - np.eye(h)).max() < 1e-13
    assert np.abs(X1.T @ X2 - X2.T @ X1).max() < 1e-13
    A = jsym.dense_from_blocks(A11, A12)
    assert np.abs(np.linalg.eigvalsh(A) - np.sort(np.concatenate([lam, lam]))).max() < 1e-13
    assert np.abs(A11 - A11.conj().T).max() < 1e-15 and np.abs(A12 + A12.T).max() == 0.0


@pytest.mark.parametrize("which", ["lowest", "largest"])
def test_pair_eigenvalues_known_spectrum(which):
    """brute() on a Case A matrix returns the planted Lambda, once per pair,
    ascending for the lowest end and descending for the largest end; the
    in-pair gap is at rounding level.  A spectrum with one planted value
    repeated in two pairs keeps both copies."""
    A11, A12, lam, _ = inputs.known_spectrum(8, 200)
    pairs, gap = jsym.brute(jsym.dense_from_blocks(A11, A12), which)
    want = lam if which == "lowest" else lam[::-1]
    assert np.abs(pairs - want).max() < 1e-13
    assert gap < 1e-13
    lam2 = np.linspace(0.1, 0.9, 50)
    lam2[7] = lam2[8]   # two distinct pairs with one eigenvalue (multiplicity 4)
    A11, A12, l2, _ = inputs.known_spectrum(9, 100, lam=lam2)
    pairs, _ = jsym.brute(jsym.dense_from_blocks(A11, A12), which)
    want = np.sort(lam2) if which == "lowest" else np.sort(lam2)[::-1]
    assert np.abs(pairs - want).max() < 1e-13


# ---------------------------------------------------------------- TRLAN-JSYM
def _check_pairs(A, X, ev, tol):
    """Outputs: residuals, partners (A y = lambda y) and [X, J X*] orthonormal."""
    n, k = X.shape
    Y = jsym.partner(X)
    for i in range(k):
        assert np.linalg.norm(A @ X[:, i] - ev[i] * X[:, i]) < tol
        assert np.linalg.norm(A @ Y[:, i] - ev[i] * Y[:, i]) < tol
    UU = np.concatenate([X, Y], axis=1)
    assert np.abs(UU.conj().T @ UU - np.eye(2 * k)).max() < 1e-12
    h = n // 2
    X1, X2 = X[:h], X[h:]
    assert np.abs(X1.T @ X2 - X2.T @ X1).max() < 1e-12


def test_trlan_dense_c1_vs_brute():
    """Dense n=200, 10 lowest pairs, m=40, mwin=20, tol 1e-10."""
    A = _dense(1, 100)
    ref, _ = jsym.brute(A)
    out = trlan.trlan_jsym(lambda v: A @ v, 200, 10, 20, 40, 1e-10)
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - ref[:10]).max() / np.abs(ref[:10]).max() < 1e-10
    assert (out["res"] < 1e-10).all()
    _check_pairs(A, out["X"], out["ev"], 1e-10)


def test_trlan_casea_largest_known_spectrum():
    A11, A12, lam, _ = inputs.known_spectrum(8, 400)
    A = jsym.dense_from_blocks(A11, A12)
    out = trlan.trlan_jsym(lambda v: A @ v, 400, 10, 20, 50, 1e-12, which="largest")
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - lam[::-1][:10]).max() < 1e-12
    _check_pairs(A, out["X"], out["ev"], 1e-12)


def test_trlan_stencil_vs_brute():
    L = (3, 3, 3, 3)
    U, B = inputs.stencil_links(4, L)
    A = jsym.stencil_dense(U, B, L)
    ref, _ = jsym.brute(A)
    n = A.shape[0]
    out = trlan.trlan_jsym(lambda v: jsym.stencil_apply(U, B, L, v), n, 12, 24, 60, 1e-10)
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - ref[:12]).max() < 1e-10 * np.abs(ref).max()
    _check_pairs(A, out["X"], out["ev"], 1e-10)


def test_trlan_constant_links_closed_form_random_start():
    """Translation-invariant stencil with a random start (all-ones lies in the
    k = 0 sector); the lowest pairs match the Fourier closed form."""
    L = (4, 4, 4, 4)
    Uc, B, U = inputs.constant_links(6, L)
    n = 2 * 256 * 4
    cf, _ = jsym.pair_eigenvalues(jsym.constant_link_spectrum(Uc, B, L))
    out = trlan.trlan_jsym(lambda v: jsym.stencil_apply(U, B, L, v), n, 8, 16, 48, 1e-10,
                           v1=inputs.random_start(7, n))
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - cf[:8]).max() < 1e-10 * np.abs(cf).max()


def test_first_step_closed_form():
    """With v_1 = ones/sqrt(n): alpha_1 = (1/n) sum_ij A_ij and
    beta_1 = ||(I - v_1 v_1^H) A v_1|| (the W-projection removes nothing by
    Lemma 1)."""
    A = _dense(5, 50)
    n = 100
    out = trlan.trlan_jsym(lambda v: A @ v, n, 4, 8, 20, 1e-10, trace_cap=1)
    v1 = np.ones(n) / math.sqrt(n)
    a1 = A.sum().real / n
    r = A @ v1 - a1 * v1
    assert abs(out["alpha"][0] - a1) < 1e-13 * abs(a1)
    assert abs(out["beta"][0] - np.linalg.norm(r)) < 1e-13 * np.linalg.norm(r)


def test_invariants_after_every_restart():
    """Cor. 1/2: V^H V = I, V^H W = 0, V^H A W = 0 (W = J V^*), and the
    Krylov-Schur relation A V_k = V_k diag(theta) + v_{k+1} s^T on decoupled
    and coupled rows (Sec. 2, thick restart)."""
    A = _dense(1, 100)
    seen = []

    def check(V, T, k):
        Vk = V[:, :k + 1]
        W = jsym.partner(Vk)
        assert np.abs(Vk.conj().T @ Vk - np.eye(k + 1)).max() < 1e-12
        assert np.abs(Vk.conj().T @ W).max() < 1e-12
        assert np.abs(Vk.conj().T @ (A @ W)).max() < 1e-11
        theta = np.diag(T)[:k]
        s = T[k, :k]
        R = A @ V[:, :k] - V[:, :k] * theta[None, :] - np.outer(V[:, k], s)
        assert np.linalg.norm(R, axis=0).max() < 1e-9
        seen.append(k)

    out = trlan.trlan_jsym(lambda v: A @ v, 200, 10, 20, 40, 1e-10, on_cycle=check)
    assert out["status"] == "ok" and len(seen) == out["n_conv"] - 1 and len(seen) >= 2


@pytest.mark.parametrize("nev,mwin,m", [(10, 20, 40), (5, 10, 30), (8, 16, 50)])
def test_mv_count_bounds(nev, mwin, m):
    """eq. MVcost: m + (m-mwin-nev)(Nconv-1) <= N_MV <= m + (m-mwin)(Nconv-1)
    (the bounds are attained at Nconv = 1, so they are non-strict)."""
    A = _dense(2, 120)
    out = trlan.trlan_jsym(lambda v: A @ v, 240, nev, mwin, m, 1e-10)
    nc, nmv = out["n_conv"], out["n_mv"]
    assert out["status"] == "ok"
    assert m + (m - mwin - nev) * (nc - 1) <= nmv <= m + (m - mwin) * (nc - 1)


def test_standard_trlan_finds_each_pair_twice():
    """Without the W-projections (standard TRLAN, Sec. 3) a doubled nev finds
    each eigenvalue twice; with them each pair appears once."""
    A = _dense(1, 60)
    ref, _ = jsym.brute(A)
    std = trlan.trlan_jsym(lambda v: A @ v, 120, 8, 16, 60, 1e-10, jsym=False)
    assert std["status"] == "ok"
    assert np.abs(std["ev"][0::2] - ref[:4]).max() < 1e-9
    assert np.abs(std["ev"][1::2] - ref[:4]).max() < 1e-9
    js = trlan.trlan_jsym(lambda v: A @ v, 120, 8, 16, 30, 1e-10)
    assert np.abs(js["ev"] - ref[:8]).max() < 1e-9


def test_exhausted_half_space_converges():
    """m = n/2 spans the whole J-half Krylov space (Sec. 2): one cycle gives
    the exact pairs."""
    A = _dense(9, 32)
    ref, _ = jsym.brute(A)
    out = trlan.trlan_jsym(lambda v: A @ v, 64, 8, 16, 32, 1e-8)
    assert out["status"] == "ok" and out["n_conv"] == 1
    assert np.abs(out["ev"] - ref[:8]).max() < 1e-10


def test_breakdown_on_invariant_start():
    """All-ones on the constant-link stencil lies in the k = 0 Fourier sector
    (an 8-dimensional invariant subspace): breakdown is reported."""
    L = (3, 3, 3, 3)
    Uc, B, U = inputs.constant_links(6, L)
    n = 2 * 81 * 4
    out = trlan.trlan_jsym(lambda v: jsym.stencil_apply(U, B, L, v), n, 8, 16, 40, 1e-10)
    assert out["status"] == "breakdown"


def _batched_problem(seed, index):
    """Problem `index` of the 512-problem batched recipe, without keeping the
    others in memory."""
    rng, n = inputs.batched_sizes(seed)
    for i in range(index + 1):
        A11, A12 = inputs.dense_jsym(rng, int(n[i]) // 2)
    return jsym.dense_from_blocks(A11, A12)


def test_relative_tolerance_keeps_converged_pairs():
    """With tol_relative the scale is a running maximum of |theta|: a pair
    decoupled as converged (its coupling set to zero, Alg. 1) is frozen, so it
    must never leave the converged set.  Problem 331 of the batched recipe
    (n = 580) has a pair whose residual sits at 1e-5 max|theta|; a per-cycle
    scale dropped it at the fourth cycle."""
    A = _batched_problem(3, 331).astype(np.complex64).astype(np.complex128)
    ref, _ = jsym.brute(A)
    out = trlan.trlan_jsym(lambda v: A @ v, A.shape[0], 8, 16, 32, 1e-5, "lowest",
                           np.ones(A.shape[0], complex), max_cycles=60, tol_relative=True,
                           record_history=True)
    assert out["status"] == "ok"
    assert np.abs(np.sort(out["ev"]) - ref[:8]).max() < 1e-5 * np.abs(ref).max()
    prev = np.zeros(0)
    for h in out["history"]:
        now = h["ev"][:h["icnv"]]
        for e in prev:
            assert np.abs(now - e).min() < 1e-12 * abs(e)
        prev = now


def test_invalid_parameters():
    A = _dense(1, 10)
    f = lambda v: A @ v
    with pytest.raises(ValueError):
        trlan.trlan_jsym(f, 20, 2, 4, 11, 1e-10)     # m > n/2
    with pytest.raises(ValueError):
        trlan.trlan_jsym(f, 20, 5, 4, 8, 1e-10)      # nev > mwin
    with pytest.raises(ValueError):
        trlan.trlan_jsym(f, 20, 2, 8, 8, 1e-10)      # mwin >= m


def test_table1_caseA_counts_in_published_range():
    """Table 1 (Case A): our own random draws of the recipe at n=2000, largest,
    tol 1e-13, (nev, mwin, m) = (10, 20, 50) land inside the printed
    [min, max] N_conv and N_MV ranges (statistical: one matrix)."""
    rows = json.load(open(os.path.join(GOLDEN, "table1_caseA.json")))["rows"]
    row = [r for r in rows if r[0] == "TRLAN-JSYM" and r[1:4] == [10, 20, 50]][0]
    for seed in (11,):
        A11, A12, lam, _ = inputs.known_spectrum(seed, 2000)
        A = jsym.dense_from_blocks(A11, A12)
        out = trlan.trlan_jsym(lambda v: A @ v, 2000, 10, 20, 50, 1e-13, which="largest")
        assert out["status"] == "ok"
        assert np.abs(out["ev"] - lam[::-1][:10]).max() < 1e-12
        assert row[4] <= out["n_conv"] <= row[6]
        assert row[7] <= out["n_mv"] <= row[9]


def test_standard_trlan_can_miss_partners():
    """Case A, n=2000, seed 12, the ten largest: the standard method converges
    before the second copy of any pair has entered its Krylov space (one
    direction per eigenspace for a single start vector, up to rounding), and
    returns ten distinct eigenvalues; the J-restricted method returns the five
    largest pairs once each, which is what it is built to do (Sec. 3)."""
    A11, A12, lam, _ = inputs.known_spectrum(12, 2000)
    A = jsym.dense_from_blocks(A11, A12)
    std = trlan.trlan_jsym(lambda v: A @ v, 2000, 10, 20, 200, 1e-13, which="largest", jsym=False)
    top = lam[::-1]
    assert std["status"] == "ok"
    assert np.abs(np.sort(std["ev"])[::-1] - top[:10]).max() < 1e-12
    js = trlan.trlan_jsym(lambda v: A @ v, 2000, 5, 10, 100, 1e-13, which="largest")
    assert js["status"] == "ok" and np.abs(js["ev"] - top[:5]).max() < 1e-12
