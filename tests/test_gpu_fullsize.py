"""Whole solves at the full 16^4 stencil shape (n = 524288, 100 lowest pairs,
m = 300, mwin = 150) pinned to results that do not come from the GPU:

* the constant-link stencil, whose spectrum is the Fourier closed form
  (`jsym.constant_link_spectrum`), in FP64 (tol 1e-10) and mixed (tol 1e-5);
* residuals of x and of its partner J x^* through the oracle's matrix-free
  stencil (FP64 operator), on a sample of the returned pairs;
* Cor. 1 and 2 on the returned vectors: X^H X = I, X^T J^T X = O (the
  partners are orthogonal to X), X^H A J X^* = O;
* the Lanczos decomposition of the GPU basis after one and after two outer
  iterations (the second one starting from a thick restart): V^H V = I,
  V^T J^T V = O and the Krylov relation A V_m = V_{m+1} Tbar, for both
  readings of the norm b0 in the first sqrt(2) test of Alg. 2.
"""
import numpy as np
import pytest

from paper_2001_07428_amd import inputs
from oracle import jsym

from gpu_util import cdt, say, to_dev, to_np

pytestmark = pytest.mark.gpu

L16 = (16, 16, 16, 16)
N16 = 2 * 16 ** 4 * 4
U32 = 2.0 ** -24      # unit roundoff of the FP32 storage
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return J.Context(0)


def _abs_rowsum_bound(U, B, diag=inputs.STENCIL_DIAG, scale=inputs.STENCIL_A12_SCALE):
    """An upper bound on || |A| ||_2 (|A| entrywise) of the stencil: the
    largest absolute row sum of |A| (|A| is symmetric, so ||.||_2 <= ||.||_inf),
    summed term by term from the operator's definition."""
    row_u = np.abs(U).sum(axis=-1).max() + np.abs(U).sum(axis=-2).max()   # U(x) and U(x-mu)^H
    row_b = np.abs(B).sum(axis=-1).max() + np.abs(B).sum(axis=-2).max()   # B and B^T
    return abs(diag) + 4 * (row_u + scale * row_b)


def _sample_residuals(U, B, L, X, ev, idx):
    """||A x - ev x|| and ||A y - ev y|| (y = J x^*) with the oracle's FP64
    stencil on the columns idx of X (rows = vectors); also A y per column."""
    rx, ry, Ay = [], [], []
    for i in idx:
        x = X[i].astype(np.complex128)
        y = jsym.partner(x)
        ax = jsym.stencil_apply(U, B, L, x)
        ay = jsym.stencil_apply(U, B, L, y)
        rx.append(np.linalg.norm(ax - ev[i] * x))
        ry.append(np.linalg.norm(ay - ev[i] * y))
        Ay.append(ay)
    return np.array(rx), np.array(ry), np.array(Ay)


@pytest.mark.parametrize("mixed", [False, True])
def test_constant_links_16_4_closed_form(ctx, mixed):
    """The 100 lowest pairs of the 16^4 constant-link stencil (random start)
    equal the Fourier closed form: relative eigenvalue error below 1e-10
    (FP64) / 1e-5 (mixed)."""
    from paper_2001_07428_amd import jlanczos as J
    say("constant links 16^4", "mixed" if mixed else "fp64")
    Uc, B, U = inputs.constant_links(6, L16)
    cf, _ = jsym.pair_eigenvalues(jsym.constant_link_spectrum(Uc, B, L16))
    nev, m, mwin = 100, 300, 150
    tol = 1e-5 if mixed else 1e-10
    op = J.jl_op_create_stencil(ctx, L16, to_dev(U, cdt(mixed)), to_dev(B, cdt(mixed)))
    v1 = to_dev(inputs.random_start(7, N16), cdt(mixed))
    out = J.jl_solve(op, nev, m, mwin, tol, v1=v1)
    print(f"  cycles {out.stats['cycles']} n_mv {out.stats['n_mv']} "
          f"gs_passes {out.stats['gs_passes']}", flush=True)
    assert out.status == J.JL_OK, out.stats
    ref = cf[:nev]
    relerr = np.abs(out.evals - ref).max() / np.abs(ref).max()
    print(f"  max rel eigenvalue error vs closed form {relerr:.2e}", flush=True)
    assert relerr < (1e-5 if mixed else 1e-10)
    assert (out.res < tol).all()
    X = to_np(out.X)
    # rounding of the operator in the storage type moves a residual by at most
    # ||A - fl(A)||_2 <= u_s || |A| ||_2 (x itself is the stored vector)
    us = U32 if mixed else U64
    dres = 2.0 * us * _abs_rowsum_bound(U, B) + 1e-13
    idx = list(range(0, nev, 10))
    rx, ry, Ay = _sample_residuals(U, B, L16, X, out.evals, idx)
    print(f"  oracle residuals x {rx.max():.2e} Jx* {ry.max():.2e}; "
          f"|res - oracle| {np.abs(rx - out.res[idx]).max():.2e} (bound {dres:.1e})", flush=True)
    assert (rx < tol + dres).all() and (ry < tol + dres).all()
    assert np.abs(rx - out.res[idx]).max() <= dres
    # Cor. 1 and 2 on the returned vectors
    Xc = X.T.astype(np.complex128)                 # n x nev
    Y = jsym.partner(Xc)
    otol = 1e-5 if mixed else 1e-12
    g = np.abs(Xc.conj().T @ Xc - np.eye(nev)).max()
    w = np.abs(Xc.conj().T @ Y).max()              # X^H J X^* = -(X^T J^T X)^*
    print(f"  ||X^H X - I||_max {g:.2e}  ||X^H J X*||_max {w:.2e}", flush=True)
    assert g < otol and w < otol
    xay = np.abs(Xc.conj().T @ Ay.T).max()         # X^H A (J x_i^*) for the sampled i
    assert xay < tol + dres + otol * _abs_rowsum_bound(U, B)


def _decomposition_errors(U, B, L, Vdev, T, meff, cols):
    """||V^H V - I||_max, ||V^T J^T V||_max over the meff + 1 basis vectors,
    and max_j ||A v_j - V_{m+1} Tbar e_j|| over the sampled columns j.  The
    Gram matrices are complex128 library products (torch) of the exported
    basis, the Krylov relation uses the oracle's FP64 stencil."""
    import torch
    Vt = Vdev[:meff + 1].to(torch.complex128)      # rows = basis vectors
    h = Vt.shape[1] // 2
    W = torch.cat([-Vt[:, h:].conj(), Vt[:, :h].conj()], dim=1)    # rows = J v^*
    Vh = Vt.conj().resolve_conj()
    G = torch.mm(Vh, Vt.transpose(0, 1))
    orth = (G - torch.eye(meff + 1, dtype=G.dtype, device=G.device)).abs().max().item()
    jorth = torch.mm(Vh, W.transpose(0, 1)).abs().max().item()
    Vc = to_np(Vt).T                               # n x (meff + 1)
    del Vt, Vh, W, G
    Tl = T[:meff + 1, :meff]
    Tm = np.tril(Tl[:meff]) + np.tril(Tl[:meff], -1).T      # symmetric T_m
    Tbar = np.vstack([Tm, Tl[meff:meff + 1]])               # row m: t_{m+1,m} e_m^T
    kry = 0.0
    for j in cols:
        r = jsym.stencil_apply(U, B, L, Vc[:, j]) - Vc @ Tbar[:, j]
        kry = max(kry, np.linalg.norm(r))
    return orth, jorth, kry


@pytest.mark.parametrize("b0_rule", [0, 1])
@pytest.mark.parametrize("mixed", [False, True])
def test_basis_decomposition_16_4(ctx, mixed, b0_rule):
    """The Lanczos basis the GPU builds at 16^4 (random links, all-ones start)
    after the first iteration and after the second (thick restart, 150 kept
    Ritz vectors and v_{m+1}): V^H V = I and V^T J^T V = O (Cor. 1), and
    A V_m = V_{m+1} Tbar up to the Gram-Schmidt coefficients that Alg. 2 does
    not keep in T (rounding level).  b0_rule 1 takes the sqrt(2) test as
    Alg. 2 prints it and so runs more second passes."""
    from paper_2001_07428_amd import jlanczos as J
    say("basis decomposition 16^4", "mixed" if mixed else "fp64", "b0_rule", b0_rule)
    U, B = inputs.stencil_links(4, L16)
    nev, m, mwin = 100, 300, 150
    tol = 1e-5
    us = U32 if mixed else U64
    anorm = _abs_rowsum_bound(U, B)
    op = J.jl_op_create_stencil(ctx, L16, to_dev(U, cdt(mixed)), to_dev(B, cdt(mixed)))
    for cyc in (1, 2):
        out = J.jl_solve(op, nev, m, mwin, tol, max_cycles=cyc, basis_cycle=cyc, b0_rule=b0_rule)
        assert out.status == J.JL_NOT_CONVERGED and out.stats["cycles"] == cyc
        orth, jorth, kry = _decomposition_errors(U, B, L16, out.basis, out.T, m,
                                                 [0, 1, 150, 151, 299])
        out.basis = None
        passes = out.stats["gs_passes"] / out.stats["n_mv"]
        print(f"  iteration {cyc}: ||V^H V - I|| {orth:.2e}  ||V^T J^T V|| {jorth:.2e}  "
              f"Krylov relation {kry:.2e}  passes/step {passes:.3f}", flush=True)
        # orthogonality: each stored vector carries one rounding to the storage
        # type (u_s / sqrt(n) per inner product) plus what the Gram-Schmidt
        # leaves; gate at 64 u_s for FP32 storage, 1e-12 for FP64
        otol = 64 * U32 if mixed else 1e-12
        assert orth < otol and jorth < otol
        # Krylov relation: apply rounding (u_s || |A| || per vector) plus the
        # discarded Gram-Schmidt coefficients (of the order of the loss of
        # orthogonality times ||A||)
        assert kry < 64 * us * anorm + 16 * otol * anorm
        if b0_rule == 1:
            assert out.stats["gs_passes"] > out.stats["n_mv"]


@pytest.mark.parametrize("b0_rule", [0, 1])
def test_basis_decomposition_fp64_long(ctx, b0_rule):
    """As test_basis_decomposition_16_4 in FP64 on a 16^3 x 32 lattice (2^19
    pairs, where the FP64 inner products stage u in LDS and fuse the local
    three-term step), 20 pairs, m = 60, mwin = 30."""
    from paper_2001_07428_amd import jlanczos as J
    L = (16, 16, 16, 32)
    say("basis decomposition fp64", L, "b0_rule", b0_rule)
    U, B = inputs.stencil_links(4, L)
    nev, m, mwin = 20, 60, 30
    anorm = _abs_rowsum_bound(U, B)
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, cdt(False)), to_dev(B, cdt(False)))
    for cyc in (1, 2):
        out = J.jl_solve(op, nev, m, mwin, 1e-10, max_cycles=cyc, basis_cycle=cyc, b0_rule=b0_rule)
        assert out.status == J.JL_NOT_CONVERGED and out.stats["cycles"] == cyc
        orth, jorth, kry = _decomposition_errors(U, B, L, out.basis, out.T, m, [0, 1, 30, 31, 59])
        out.basis = None
        print(f"  iteration {cyc}: ||V^H V - I|| {orth:.2e}  ||V^T J^T V|| {jorth:.2e}  "
              f"Krylov relation {kry:.2e}", flush=True)
        assert orth < 1e-12 and jorth < 1e-12
        assert kry < 64 * U64 * anorm + 16 * 1e-12 * anorm
