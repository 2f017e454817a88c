"""Invert mode on the device (Alg. 1 and 2, invert branches; A^-1 v_j by
conjugate gradients, Sec. 4.2) against the FP64 oracle's invert mode on the
same seeded inputs, through the C ABI."""
import numpy as np
import pytest

from paper_2001_07428_amd import inputs
from oracle import cg, jsym, trlan

from gpu_util import cdt, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return J.Context(0)


def _cg_solve(apply, rtol=1e-14):
    def solve(v):
        x, _, ok, _ = cg.cg(apply, v, rtol, 20000)
        assert ok
        return x
    return solve


def _check_pairs(apply, X, ev, tol_res, tol_orth):
    Y = jsym.partner(X.T)
    for i in range(X.shape[0]):
        assert np.linalg.norm(apply(X[i]) - ev[i] * X[i]) < tol_res
        assert np.linalg.norm(apply(Y[:, i]) - ev[i] * Y[:, i]) < tol_res
    UU = np.concatenate([X.T, Y], axis=1)
    assert np.abs(UU.conj().T @ UU - np.eye(UU.shape[1])).max() < tol_orth


def test_invert_dense_casea_fp64(ctx):
    """Case A, n=400, Lambda uniform on (0, 1): the 10 lowest pairs, m=50,
    mwin=20, tol 1e-11 (absolute), FP64."""
    from paper_2001_07428_amd import jlanczos as J
    say("invert dense casea n400 fp64")
    A11, A12, lam, _ = inputs.known_spectrum(8, 400)
    A = jsym.dense_from_blocks(A11, A12)
    f = lambda v: A @ v
    ref = trlan.trlan_jsym(f, 400, 10, 20, 50, 1e-11, mode="invert", solve=_cg_solve(f))
    assert ref["status"] == "ok"
    op = J.jl_op_create_dense(ctx, to_dev(A11, cdt(False)), to_dev(A12, cdt(False)))
    out = J.jl_solve(op, 10, 50, 20, 1e-11, invert=True, cg_tol=1e-14)
    assert out.status == J.JL_OK
    assert np.abs(out.evals - ref["ev"]).max() < 1e-11
    assert np.abs(out.evals - lam[:10]).max() < 1e-11
    assert (out.res < 1e-11).all()
    assert abs(out.stats["n_mv"] - ref["n_mv"]) <= 30   # one cycle's steps at most
    assert out.stats["cg_iters"] >= out.stats["n_mv"]
    assert out.stats["cg_unconverged"] == 0
    _check_pairs(f, to_np(out.X), out.evals, 1e-11, 1e-12)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (3, 4, 2, 5)])
def test_invert_stencil_fp64_vs_oracle(ctx, L):
    from paper_2001_07428_amd import jlanczos as J
    say("invert stencil fp64", L)
    U, B = inputs.stencil_links(4, L)
    n = 2 * int(np.prod(L)) * 4
    f = lambda v: jsym.stencil_apply(U, B, L, v)
    ref = trlan.trlan_jsym(f, n, 8, 16, 40, 1e-10, mode="invert", solve=_cg_solve(f))
    assert ref["status"] == "ok"
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, cdt(False)), to_dev(B, cdt(False)))
    out = J.jl_solve(op, 8, 40, 16, 1e-10, invert=True, cg_tol=1e-13)
    assert out.status == J.JL_OK
    assert np.abs(out.evals - ref["ev"]).max() < 1e-10 * ref["ev"].max()
    _check_pairs(f, to_np(out.X), out.evals, 1e-10, 1e-12)
    # the lowest of the normal mode agree
    nrm = J.jl_solve(op, 8, 40, 16, 1e-10)
    assert np.abs(out.evals - nrm.evals).max() < 1e-10 * ref["ev"].max()


def test_invert_stencil_mixed(ctx):
    """FP32 storage: CG to 1e-6, pairs to a relative 1e-5."""
    from paper_2001_07428_amd import jlanczos as J
    L = (4, 4, 4, 4)
    say("invert stencil mixed", L)
    U, B = inputs.stencil_links(4, L)
    n = 2 * 256 * 4
    f = lambda v: jsym.stencil_apply(U, B, L, v)
    ref = trlan.trlan_jsym(f, n, 8, 16, 40, 1e-10, mode="invert", solve=_cg_solve(f))
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, cdt(True)), to_dev(B, cdt(True)))
    out = J.jl_solve(op, 8, 40, 16, 1e-5, invert=True, cg_tol=1e-6, tol_relative=True)
    assert out.status == J.JL_OK
    assert np.abs(out.evals - ref["ev"]).max() < 1e-5 * ref["ev"].max()
    X = to_np(out.X).astype(np.complex128)
    _check_pairs(f, X, out.evals, 2e-4, 1e-5)


def test_invert_standard_mode_finds_pairs_twice(ctx):
    from paper_2001_07428_amd import jlanczos as J
    say("invert standard dense casea n200")
    A11, A12, lam, _ = inputs.known_spectrum(21, 200)
    A = jsym.dense_from_blocks(A11, A12)
    op = J.jl_op_create_dense(ctx, to_dev(A11, cdt(False)), to_dev(A12, cdt(False)))
    out = J.jl_solve(op, 8, 40, 16, 1e-11, invert=True, standard=True, cg_tol=1e-14)
    assert out.status == J.JL_OK
    assert np.abs(np.sort(out.evals) - np.repeat(lam[:4], 2)).max() < 1e-11


def test_invert_rejects_negative_definite(ctx):
    """p^H A p < 0 at the first CG step: an error, every kernel exits."""
    from paper_2001_07428_amd import jlanczos as J
    say("invert negative definite")
    A11, A12, _, _ = inputs.known_spectrum(22, 100, -np.linspace(0.5, 1.0, 50))
    op = J.jl_op_create_dense(ctx, to_dev(A11, cdt(False)), to_dev(A12, cdt(False)))
    with pytest.raises(J.JLError, match="positive definite"):
        J.jl_solve(op, 2, 10, 4, 1e-10, invert=True)


def test_invert_cg_cap_is_reported(ctx):
    from paper_2001_07428_amd import jlanczos as J
    say("invert cg cap")
    A11, A12, _, _ = inputs.known_spectrum(23, 200, np.linspace(1e-3, 1.0, 100))
    op = J.jl_op_create_dense(ctx, to_dev(A11, cdt(False)), to_dev(A12, cdt(False)))
    out = J.jl_solve(op, 4, 20, 8, 1e-12, invert=True, cg_maxit=3, max_cycles=2)
    assert out.stats["cg_max_iters"] == 3
    assert out.stats["cg_unconverged"] > 0
    assert out.stats["cg_iters"] == 3 * out.stats["n_mv"]


def test_invert_rejected_by_batch(ctx):
    from paper_2001_07428_amd import jlanczos as J
    A11, A12 = inputs.dense_jsym(3, 40)
    with pytest.raises(J.JLError):
        J.Batch(ctx, [to_dev(A11, cdt(False))], [to_dev(A12, cdt(False))], 2, 10, 4, 1e-8,
                invert=True)


@pytest.mark.parametrize("mixed", [False, True])
def test_invert_stencil_per_site_B(ctx, mixed):
    """Per-site B through the fused CG direction (both stencil kernels)."""
    from paper_2001_07428_amd import jlanczos as J
    L = (4, 4, 4, 4)
    say("invert stencil per-site B", mixed)
    U, B = inputs.stencil_links(9, L, b_per_site=True)
    n = 2 * 256 * 4
    f = lambda v: jsym.stencil_apply(U, B, L, v)
    ref = trlan.trlan_jsym(f, n, 6, 12, 36, 1e-10, mode="invert", solve=_cg_solve(f))
    assert ref["status"] == "ok"
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, cdt(mixed)), to_dev(B, cdt(mixed)))
    tol, cgt = (1e-5, 1e-7) if mixed else (1e-10, 1e-13)
    out = J.jl_solve(op, 6, 36, 12, tol, invert=True, cg_tol=cgt, tol_relative=mixed)
    assert out.status == J.JL_OK
    assert np.abs(out.evals - ref["ev"]).max() < (1e-5 if mixed else 1e-10) * ref["ev"].max()


def test_invert_large_fp32_lattice(ctx):
    """(24, 24, 16, 16): FP32 takes the plane-pair brick kernel with the
    fused CG direction.  The pairs agree with the normal mode on the GPU (its
    parity is tested against the oracle) and their residuals, checked with
    the oracle's operator, are below the tolerance."""
    from paper_2001_07428_amd import jlanczos as J
    L = (24, 24, 16, 16)
    say("invert large fp32", L)
    U, B = inputs.stencil_links(12, L)
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, cdt(True)), to_dev(B, cdt(True)))
    inv = J.jl_solve(op, 4, 24, 8, 1e-5, invert=True, cg_tol=1e-7, tol_relative=True)
    nrm = J.jl_solve(op, 4, 24, 8, 1e-5, tol_relative=True, max_cycles=2000)
    assert inv.status == J.JL_OK and nrm.status == J.JL_OK
    assert np.abs(inv.evals - nrm.evals).max() < 3e-4
    X = to_np(inv.X).astype(np.complex128)
    for i in range(4):
        r = jsym.stencil_apply(U, B, L, X[i]) - inv.evals[i] * X[i]
        assert np.linalg.norm(r) < 2e-4
