"""The Case B operator on the device (Sec. 4.2: A = D D^H, J = C gamma_5, in the
canonical layout [psi_0; psi_2 | psi_1; psi_3]) against the FP64 oracle's
dense definition and matrix-free form, and solves with it, through the C ABI."""
import numpy as np
import pytest

from paper_2001_07428_amd import inputs
from oracle import jsym, tek, trlan

from gpu_util import cdt, say, to_dev, to_np

pytestmark = pytest.mark.gpu

KAPPA = 0.12


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return J.Context(0)


def _op(ctx, Us, mixed, kappa=KAPPA):
    from paper_2001_07428_amd import jlanczos as J
    return J.jl_op_create_tek(ctx, to_dev(Us, cdt(mixed)), kappa)


def _ref_apply(Us, v, kappa=KAPPA):
    """A v in the canonical layout from the oracle's matrix-free form."""
    N = Us.shape[1]
    na = N * N - 1
    return tek.to_canonical(tek.apply_A(Us, kappa, tek.from_canonical(v, na), entries=True), na)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("N", [2, 3, 5])
@pytest.mark.parametrize("mixed", [False, True])
def test_tek_apply_vs_dense_definition(ctx, N, mixed):
    from paper_2001_07428_amd import jlanczos as J
    say("tek apply dense", N, mixed)
    Us = inputs.haar_su(10 + N, N, 4)
    na = N * N - 1
    A = tek.dense_A(Us, KAPPA)
    P = tek.canonical_matrix(np.kron(tek.J4.real, np.eye(na)))
    Ac = P.T @ A @ P
    X = inputs.cn(np.random.default_rng(N), (2, 4 * na))
    op = _op(ctx, Us, mixed)
    Y = to_np(J.jl_op_apply(op, to_dev(X, cdt(mixed))))
    for r in range(2):
        assert _rel(Y[r], Ac @ X[r]) < (2e-6 if mixed else 1e-13)


@pytest.mark.parametrize("N", [17, 64, 65, 100])
@pytest.mark.parametrize("mixed", [False, True])
def test_tek_apply_vs_matrix_free(ctx, N, mixed):
    """Across one and several 64-wide product tiles, with ragged edges."""
    from paper_2001_07428_amd import jlanczos as J
    say("tek apply", N, mixed)
    Us = inputs.haar_su(20 + N, N, 4)
    x = inputs.cn(np.random.default_rng(N), (4 * (N * N - 1),))
    op = _op(ctx, Us, mixed)
    y = to_np(J.jl_op_apply(op, to_dev(x, cdt(mixed))))
    assert _rel(y, _ref_apply(Us, x)) < (1e-5 if mixed else 1e-13)


@pytest.mark.parametrize("mixed", [False, True])
def test_tek_apply_full_size_289(ctx, mixed):
    """N = 289 (n = 334080, the paper's Case B size), every output."""
    from paper_2001_07428_amd import jlanczos as J
    say("tek apply 289", mixed)
    Us = inputs.haar_su(289, 289, 4)
    x = inputs.cn(np.random.default_rng(5), (4 * (289 * 289 - 1),))
    op = _op(ctx, Us, mixed)
    y = to_np(J.jl_op_apply(op, to_dev(x, cdt(mixed))))
    assert _rel(y, _ref_apply(Us, x)) < (2e-5 if mixed else 1e-12)


def test_tek_hermitian_and_J_symmetric_on_device(ctx):
    from paper_2001_07428_amd import jlanczos as J
    say("tek symmetry")
    N = 9
    Us = inputs.haar_su(31, N, 4)
    n = 4 * (N * N - 1)
    rng = np.random.default_rng(7)
    x, y = inputs.cn(rng, (n,)), inputs.cn(rng, (n,))
    op = _op(ctx, Us, False)
    Ax = to_np(J.jl_op_apply(op, to_dev(x, cdt(False))))
    Ay = to_np(J.jl_op_apply(op, to_dev(y, cdt(False))))
    assert abs(np.vdot(y, Ax) - np.conj(np.vdot(x, Ay))) < 1e-12 * np.abs(Ax).sum()
    AJx = to_np(J.jl_op_apply(op, to_dev(jsym.partner(x), cdt(False))))
    assert _rel(AJx, jsym.partner(Ax)) < 1e-13


def test_tek_solve_fp64_vs_brute(ctx):
    from paper_2001_07428_amd import jlanczos as J
    say("tek solve N5")
    N = 5
    Us = inputs.haar_su(41, N, 4)
    na = N * N - 1
    A = tek.dense_A(Us, KAPPA)
    P = tek.canonical_matrix(np.kron(tek.J4.real, np.eye(na)))
    Ac = P.T @ A @ P
    ref, _ = jsym.brute(Ac)
    op = _op(ctx, Us, False)
    out = J.jl_solve(op, 6, 24, 12, 1e-10)
    assert out.status == J.JL_OK
    assert _rel(out.evals, ref[:6]) < 1e-10
    X = to_np(out.X)
    for i in range(6):
        for v in (X[i], jsym.partner(X[i])):
            assert np.linalg.norm(Ac @ v - out.evals[i] * v) < 1e-10 * ref[-1]


@pytest.mark.parametrize("mixed", [False, True])
def test_tek_solve_vs_oracle(ctx, mixed):
    """N = 17 (n = 1152), 8 lowest pairs; the oracle runs Alg. 1 on its
    matrix-free form of the same operator."""
    from paper_2001_07428_amd import jlanczos as J
    say("tek solve N17", mixed)
    N = 17
    Us = inputs.haar_su(51, N, 4)
    n = 4 * (N * N - 1)
    ref = trlan.trlan_jsym(lambda v: _ref_apply(Us, v), n, 8, 16, 40, 1e-10)
    assert ref["status"] == "ok"
    op = _op(ctx, Us, mixed)
    out = J.jl_solve(op, 8, 40, 16, 1e-5 if mixed else 1e-10, tol_relative=mixed)
    assert out.status == J.JL_OK
    assert _rel(out.evals, ref["ev"]) < (1e-5 if mixed else 1e-10)


def test_tek_invert_mode(ctx):
    """The small eigenvalues by CG, as the paper runs Case B (Sec. 4.2)."""
    from paper_2001_07428_amd import jlanczos as J
    say("tek invert N5")
    N = 5
    Us = inputs.haar_su(61, N, 4)
    na = N * N - 1
    A = tek.dense_A(Us, KAPPA)
    P = tek.canonical_matrix(np.kron(tek.J4.real, np.eye(na)))
    ref, _ = jsym.brute(P.T @ A @ P)
    op = _op(ctx, Us, False)
    out = J.jl_solve(op, 4, 20, 8, 1e-10, invert=True, cg_tol=1e-13)
    assert out.status == J.JL_OK
    assert _rel(out.evals, ref[:4]) < 1e-10


def test_tek_rejects_bad_sizes(ctx):
    from paper_2001_07428_amd import jlanczos as J
    import torch
    U1 = torch.zeros((4, 1, 1), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(J.JLError):
        J.jl_op_create_tek(ctx, U1, KAPPA)


def test_tek_standard_mode_finds_pairs_twice(ctx):
    from paper_2001_07428_amd import jlanczos as J
    say("tek standard N5")
    N = 5
    Us = inputs.haar_su(71, N, 4)
    na = N * N - 1
    A = tek.dense_A(Us, KAPPA)
    P = tek.canonical_matrix(np.kron(tek.J4.real, np.eye(na)))
    ref, _ = jsym.brute(P.T @ A @ P)
    op = _op(ctx, Us, False)
    out = J.jl_solve(op, 8, 40, 16, 1e-10, standard=True)
    assert out.status == J.JL_OK
    assert np.abs(np.sort(out.evals) - np.repeat(ref[:4], 2)).max() < 1e-10 * ref[-1]
