"""Step-level parity of the HIP kernels against the FP64 oracle / NumPy
(through the C ABI)."""
import numpy as np
import pytest

from paper_2001_07428_amd import inputs
from oracle import jsym

from gpu_util import cdt, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return J.Context(0)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ------------------------------------------------------------------ operators
@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 3, 4, 5), (3, 2, 2, 7), (8, 8, 16, 8), (6, 4, 16, 16),
                               (5, 8, 8, 16)])
@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("b_per_site", [False, True])
def test_stencil_apply(ctx, L, mixed, b_per_site):
    """Three columns at once, every output.  (8, 8, 16, 8) and (6, 4, 16, 16)
    have x0-planes of 1024 sites and an even L0, which the FP32 apply takes in
    plane-pair bricks; (5, 8, 8, 16) has an odd L0."""
    from paper_2001_07428_amd import jlanczos as J
    say("stencil_apply", L, mixed, b_per_site)
    U, B = inputs.stencil_links(4, L, b_per_site=b_per_site)
    n = 2 * int(np.prod(L)) * 4
    X = inputs.cn(np.random.default_rng(3), (3, n))
    dt = cdt(mixed)
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, dt), to_dev(B, dt))
    Y = to_np(J.jl_op_apply(op, to_dev(X, dt)))
    for r in range(3):
        ref = jsym.stencil_apply(U, B, L, X[r])
        assert _rel(Y[r], ref) < (2e-6 if mixed else 1e-14)


@pytest.mark.parametrize("L", [(16, 16, 16, 16), (24, 24, 16, 16)])
@pytest.mark.parametrize("mixed", [False, True])
def test_stencil_apply_large(ctx, L, mixed):
    """The benchmark's 16^4 shape and a lattice with unequal extents
    (V = 147456), every output."""
    from paper_2001_07428_amd import jlanczos as J
    say("stencil_apply large", L, mixed)
    U, B = inputs.stencil_links(4, L)
    n = 2 * int(np.prod(L)) * 4
    x = inputs.cn(np.random.default_rng(3), (1, n))
    dt = cdt(mixed)
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, dt), to_dev(B, dt))
    y = to_np(J.jl_op_apply(op, to_dev(x, dt)))[0]
    assert _rel(y, jsym.stencil_apply(U, B, L, x[0])) < (2e-6 if mixed else 1e-14)


_LINKS32 = {}


@pytest.mark.parametrize("mixed", [False, True])
def test_stencil_apply_32(ctx, mixed):
    """The 32^4 lattice of the headline configuration (n = 8388608), every
    output, in the launch configuration the solver uses."""
    from paper_2001_07428_amd import jlanczos as J
    L = (32, 32, 32, 32)
    say("stencil_apply 32^4", mixed)
    if not _LINKS32:
        _LINKS32["UB"] = inputs.stencil_links(5, L)
    U, B = _LINKS32["UB"]
    n = 2 * int(np.prod(L)) * 4
    x = inputs.cn(np.random.default_rng(11), (1, n))
    dt = cdt(mixed)
    op = J.jl_op_create_stencil(ctx, L, to_dev(U, dt), to_dev(B, dt))
    y = to_np(J.jl_op_apply(op, to_dev(x, dt)))[0]
    assert _rel(y, jsym.stencil_apply(U, B, L, x[0])) < (2e-6 if mixed else 1e-14)


@pytest.mark.parametrize("h", [100, 33, 1, 1500, 2053])
@pytest.mark.parametrize("mixed", [False, True])
def test_dense_apply(ctx, h, mixed):
    from paper_2001_07428_amd import jlanczos as J
    say("dense_apply", h, mixed)
    A11, A12 = inputs.dense_jsym(1, h)
    A = jsym.dense_from_blocks(A11, A12)
    X = inputs.cn(np.random.default_rng(4), (2, 2 * h))
    dt = cdt(mixed)
    op = J.jl_op_create_dense(ctx, to_dev(A11, dt), to_dev(A12, dt))
    Y = to_np(J.jl_op_apply(op, to_dev(X, dt)))
    for r in range(2):
        assert _rel(Y[r], A @ X[r]) < (2e-6 if mixed else 1e-14)


@pytest.mark.parametrize("mixed", [False, True])
def test_pair_vectors(ctx, mixed):
    from paper_2001_07428_amd import jlanczos as J
    say("pair_vectors", mixed)
    X = inputs.cn(np.random.default_rng(5), (4, 202))
    Y = to_np(J.jl_pair_vectors(ctx, to_dev(X, cdt(mixed))))
    ref = jsym.partner(X.T).T
    assert _rel(Y, ref) < (1e-7 if mixed else 0.0) + 1e-300
    # in place
    Xd = to_dev(X, cdt(mixed))
    J.jl_pair_vectors(ctx, Xd, Xd)
    assert _rel(to_np(Xd), ref) < (1e-7 if mixed else 0.0) + 1e-300


# ----------------------------------------------------------- reorthogonalisation
@pytest.mark.parametrize("h,ncol", [(1000, 7), (33, 5), (5000, 130), (4096, 1), (640, 0),
                                    (40000, 77), (262144, 70), (300, 2047),
                                    (4194304, 6), (1048576, 3), (1048578, 2), (1048577, 2),
                                    (2097152, 3), (2097154, 2)])
@pytest.mark.parametrize("mixed", [False, True])
def test_reorth_pass(ctx, h, ncol, mixed):
    """One block Gram-Schmidt pass against [V, W = J V^*] (Alg. 2).  The two
    long vectors take the inner-product reduction over 2 and 16 row slices
    (tiles of 64 sums, the last one ragged); the 262144-pair case's basis
    (over 256 MB) is read with non-temporal loads, as is the 32^4-sized one
    (4194304 pairs); 2047 columns is the largest basis a pass takes (its LDS
    accumulators and 128 reduction tiles).  From 1048576 pairs (even) the FP32
    inner products stage u in LDS (1048578: a last block of two pairs;
    1048577, odd, stays on the register kernel); from 2097152 pairs (even) the
    FP32 update keeps its corrections in LDS, one wavefront per 1024 pairs
    (2097154: a last block of two pairs; 4194304 with non-temporal loads).
    From 524288 pairs the FP64 inner products stage u in LDS, 2048 pairs per
    block (1048577: a last block of one pair)."""
    from paper_2001_07428_amd import jlanczos as J
    say("reorth_pass", h, ncol, mixed)
    rng = np.random.default_rng(6)
    n = 2 * h
    V = inputs.cn(rng, (ncol, n)) / np.sqrt(n)
    u = inputs.cn(rng, n)
    dt = cdt(mixed)
    Vd, ud = to_dev(V, dt), to_dev(u, dt)
    Vq, uq = to_np(Vd).astype(np.complex128), to_np(ud).astype(np.complex128)   # rounded inputs
    coef = to_np(J.jl_reorth_pass(ctx, Vd if ncol else None, ud))
    W = jsym.partner(Vq.T).T
    cv = Vq.conj() @ uq
    cw = W.conj() @ uq
    got_cv = coef[0:4 * ncol:4] + 1j * coef[1:4 * ncol:4]
    got_cw = coef[2:4 * ncol:4] + 1j * coef[3:4 * ncol:4]
    scale = np.linalg.norm(uq) * (np.abs(Vq).max() if ncol else 1.0) * np.sqrt(n)
    if ncol:
        assert np.abs(got_cv - cv).max() < 1e-13 * scale
        assert np.abs(got_cw - cw).max() < 1e-13 * scale
    assert abs(coef[4 * ncol] - np.vdot(uq, uq).real) < 1e-12 * np.vdot(uq, uq).real
    unew = uq - cv @ Vq - cw @ W
    got = to_np(ud).astype(np.complex128)
    # the update sums 2 ncol + 1 terms in the storage precision: a rounding
    # bound per element, scaled by the magnitudes of those terms (the columns
    # here are random, not orthonormal, so the coefficients are O(1)), plus one
    # unit of the reference's own rounding
    eps = 6e-8 if mixed else 1.2e-16
    mag = np.abs(uq)
    if ncol:
        mag = mag + np.abs(cv) @ np.abs(Vq) + np.abs(cw) @ np.abs(W)
    bound = 8 * eps * np.sqrt(2 * ncol + 1) * mag + eps * np.abs(uq).max()
    assert (np.abs(got - unew) <= bound).all()
    assert abs(coef[4 * ncol + 1] - np.vdot(got, got).real) < 1e-12 * max(np.vdot(got, got).real, 1e-300)


# ------------------------------------------------------------------ Ritz step
def _arrow(rng, m, k):
    """Thick-restart projected matrix: diag(theta) (k), arrow row k, then a
    tridiagonal tail; a few arrow entries are exactly zero (decoupled)."""
    T = np.zeros((m, m))
    T[np.arange(k), np.arange(k)] = np.sort(rng.standard_normal(k))
    s = rng.standard_normal(k) * 0.3
    s[::3] = 0.0
    T[k, :k] = s
    T[:k, k] = s
    a = rng.standard_normal(m - k) * 2
    b = np.abs(rng.standard_normal(m - k - 1)) + 0.1
    T[np.arange(k, m), np.arange(k, m)] = a
    T[np.arange(k + 1, m), np.arange(k, m - 1)] = b
    T[np.arange(k, m - 1), np.arange(k + 1, m)] = b
    return T


@pytest.mark.parametrize("m", [1, 2, 10, 41, 59, 60, 61, 160, 301])
@pytest.mark.parametrize("which", ["lowest", "largest"])
def test_ritz(ctx, m, which):
    """T = Z diag(lam) Z^T (Alg. 1), sorted, vs numpy eigh."""
    import torch
    from paper_2001_07428_amd import jlanczos as J
    say("ritz", m, which)
    rng = np.random.default_rng(m)
    G = rng.standard_normal((m, m))
    for T in (G + G.T, _arrow(rng, m, m // 2) if m > 3 else G + G.T):
        lam, Z = J.jl_ritz(ctx, torch.from_numpy(T).cuda(), which)
        lam, Z = to_np(lam), to_np(Z)
        ref = np.linalg.eigvalsh(T)
        if which == "largest":
            ref = ref[::-1]
        nrm = np.linalg.norm(T, 2)
        assert np.abs(lam - ref).max() < 1e-13 * nrm * max(1, np.sqrt(m) / 4)
        assert np.abs(T @ Z - Z * lam[None, :]).max() < 1e-12 * nrm
        assert np.abs(Z.T @ Z - np.eye(m)).max() < 1e-12


# -------------------------------------------------------------- restart GEMM
@pytest.mark.parametrize("h,m,k", [(1000, 37, 29), (2048, 160, 130), (50, 3, 3), (3000, 129, 1),
                                   (6144, 300, 250), (2048, 160, 80), (2048, 160, 100),
                                   (1000, 200, 50), (6144, 300, 300), (2048, 256, 208)])
@pytest.mark.parametrize("mixed", [False, True])
def test_basis_update(ctx, h, m, k, mixed):
    """V_k = V_m Z[:, :k] (Alg. 1) as a real GEMM on the interleaved basis,
    FP64 accumulation for both storage types (mixed: one final rounding).
    The k values reach every split of the columns over 128-, 64- and 32-wide
    tiles."""
    from paper_2001_07428_amd import jlanczos as J
    say("basis_update", h, m, k, mixed)
    rng = np.random.default_rng(7)
    V = inputs.cn(rng, (m, 2 * h))
    Z = rng.standard_normal((m, k))
    dt = cdt(mixed)
    Vd = to_dev(V, dt)
    import torch
    Zd = torch.from_numpy(Z).cuda()
    Y = to_np(J.jl_basis_update(ctx, Vd, Zd)).astype(np.complex128)
    Vq = to_np(Vd).astype(np.complex128)
    Zq = Z
    ref = Zq.T @ Vq
    err = np.abs(Y - ref).max() / (np.abs(Vq).max() * np.abs(Zq).sum(0).max())
    assert err < (1e-7 if mixed else 1e-14)
