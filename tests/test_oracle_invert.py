"""Pins for the invert mode of the oracle (Alg. 1 and 2, invert branches; CG
for A^-1 v, Sec. 4.2): direct solves, the finite termination of CG, the
J-equivariance of the solve, the residual-estimate identity, brute-force and
known spectra.  CPU only."""
import numpy as np
import pytest

from paper_2001_07428_amd import inputs
from oracle import cg, jsym, trlan


def _casea(seed, n, lam=None):
    A11, A12, lam, _ = inputs.known_spectrum(seed, n, lam)
    return jsym.dense_from_blocks(A11, A12), lam


# ------------------------------------------------------------------ CG
def test_cg_matches_direct_solve():
    A, lam = _casea(3, 200, np.linspace(0.5, 4.0, 100))
    b = inputs.random_start(4, 200)
    x, it, ok, hist = cg.cg(lambda v: A @ v, b, 1e-14, 1000)
    ref = np.linalg.solve(A, b)
    assert ok and it < 200
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    assert hist[-1] <= 1e-14 * hist[0]


def test_cg_finite_termination_with_three_eigenvalues():
    """The Krylov space of a matrix with three distinct eigenvalues has
    dimension three, so CG ends at the exact solution after three steps; a
    wrong alpha or beta (or a missing conjugation) does not."""
    lam = np.repeat([0.5, 1.25, 3.0], [20, 30, 30])
    A, _ = _casea(5, 160, lam)
    b = inputs.random_start(6, 160)
    x, it, ok, hist = cg.cg(lambda v: A @ v, b, 1e-13, 50)
    assert ok and it == 3
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_cg_is_J_equivariant():
    """For Hermitian J-symmetric A, A (J b^*) = J (A b)^* (eq. symmetry), and CG
    run on J b^* produces J x^* at every step (its scalars are real)."""
    A, _ = _casea(7, 120, np.linspace(0.2, 2.0, 60))
    b = inputs.random_start(8, 120)
    x1, it1, _, _ = cg.cg(lambda v: A @ v, b, 1e-12, 500)
    x2, it2, _, _ = cg.cg(lambda v: A @ v, jsym.partner(b), 1e-12, 500)
    assert it1 == it2
    assert np.abs(x2 - jsym.partner(x1)).max() <= 1e-12 * np.abs(x1).max()


def test_cg_zero_rhs():
    x, it, ok, _ = cg.cg(lambda v: v, np.zeros(10, complex), 1e-12, 10)
    assert ok and it == 0 and not x.any()


# ------------------------------------------------------------- invert mode
def test_invert_mode_casea_lowest_known_spectrum():
    """Case A, Lambda uniform on (0, 1): the lowest eigenvalues from the
    invert mode with an exact solve, each pair found once."""
    A, lam = _casea(8, 400)
    out = trlan.trlan_jsym(lambda v: A @ v, 400, 10, 20, 50, 1e-12, mode="invert",
                           solve=lambda v: np.linalg.solve(A, v))
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - lam[:10]).max() < 1e-12
    assert (out["res"] < 1e-12).all()
    # each eigenvalue once: the pairs are distinct and their partners are not among X
    assert len(np.unique(np.round(out["ev"], 10))) == 10
    X = out["X"]
    assert np.abs(X.conj().T @ jsym.partner(X)).max() < 1e-10


def test_invert_mode_with_cg_matches_exact_solve():
    A, lam = _casea(9, 300)
    stats = dict(iters=0)

    def solve(v):
        x, it, ok, _ = cg.cg(lambda u: A @ u, v, 1e-14, 5000)
        assert ok
        stats["iters"] += it
        return x

    out = trlan.trlan_jsym(lambda v: A @ v, 300, 8, 16, 40, 1e-11, mode="invert", solve=solve)
    ref = trlan.trlan_jsym(lambda v: A @ v, 300, 8, 16, 40, 1e-11, mode="invert",
                           solve=lambda v: np.linalg.solve(A, v))
    assert out["status"] == "ok" and ref["status"] == "ok"
    assert np.abs(out["ev"] - lam[:8]).max() < 1e-11
    assert np.abs(out["ev"] - ref["ev"]).max() < 1e-11
    assert stats["iters"] >= out["n_mv"]


def test_invert_residual_estimate_is_the_true_residual():
    """With an exact solve, A^-1 y = theta y + t v_{m+1} gives
    A y - (1/theta) y = -(t/theta) A v_{m+1}: the estimate c |t ev| of Alg. 1
    equals the true residual.  A huge tol accepts every pair after one cycle,
    so both are computed for all of them."""
    A, _ = _casea(10, 300, np.linspace(1.0, 2.0, 150))   # crowded for A^-1 too
    out = trlan.trlan_jsym(lambda v: A @ v, 300, 8, 10, 20, 1e3, mode="invert",
                           solve=lambda v: np.linalg.solve(A, v), record_history=True)
    est = out["history"][0]["res_est"]
    assert out["n_conv"] == 1 and (out["res"] > 1e-9).all()
    np.testing.assert_allclose(out["res"], est, rtol=1e-6)


def test_invert_mode_stencil_vs_brute():
    """Random-link stencil (positive definite for diag 8.1) with CG."""
    L = (2, 3, 2, 3)
    U, B = inputs.stencil_links(11, L)
    A = jsym.stencil_dense(U, B, L)
    ref, _ = jsym.brute(A)
    n = A.shape[0]
    assert ref[0] > 0

    def solve(v):
        x, _, ok, _ = cg.cg(lambda u: jsym.stencil_apply(U, B, L, u), v, 1e-14, 2000)
        assert ok
        return x

    out = trlan.trlan_jsym(lambda v: jsym.stencil_apply(U, B, L, v), n, 6, 12, 40, 1e-10,
                           mode="invert", solve=solve)
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - ref[:6]).max() < 1e-10 * ref[-1]


def test_invert_mode_needs_fewer_steps_at_the_dense_end():
    """Lambda uniform on (0, 1): the lowest pairs are crowded for A but well
    separated for A^-1, so the invert mode converges in far fewer steps."""
    A, lam = _casea(12, 400)
    kw = dict(which="lowest", max_cycles=400)
    nrm = trlan.trlan_jsym(lambda v: A @ v, 400, 5, 10, 30, 1e-10, **kw)
    inv = trlan.trlan_jsym(lambda v: A @ v, 400, 5, 10, 30, 1e-10, mode="invert",
                           solve=lambda v: np.linalg.solve(A, v), **kw)
    assert inv["status"] == "ok"
    assert np.abs(inv["ev"] - lam[:5]).max() < 1e-10
    assert inv["n_mv"] * 3 < nrm["n_mv"]


def test_invert_mode_relative_tolerance():
    A, lam = _casea(13, 200, np.linspace(1e-3, 1.0, 100))
    out = trlan.trlan_jsym(lambda v: A @ v, 200, 4, 8, 24, 1e-12, mode="invert",
                           solve=lambda v: np.linalg.solve(A, v), tol_relative=True)
    assert out["status"] == "ok"
    assert np.abs(out["ev"] - lam[:4]).max() < 1e-11


def test_invert_mode_parameters():
    with pytest.raises(ValueError):
        trlan.trlan_jsym(lambda v: v, 20, 2, 4, 8, 1e-8, mode="invert")
    with pytest.raises(ValueError):
        trlan.trlan_jsym(lambda v: v, 20, 2, 4, 8, 1e-8, mode="shift")
