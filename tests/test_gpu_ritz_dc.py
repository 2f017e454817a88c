"""Rayleigh-Ritz for the restart structure of T_m (divide and conquer on the
device) against numpy.linalg.eigh of the assembled matrix."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return J.Context(0)


def assemble(theta, s, alpha, beta):
    k, m = len(theta), len(theta) + len(alpha)
    T = np.zeros((m, m))
    T[np.arange(k), np.arange(k)] = theta
    T[k, :k] = s
    T[:k, k] = s
    T[np.arange(k, m), np.arange(k, m)] = alpha
    for i, b in enumerate(beta):
        T[k + i + 1, k + i] = T[k + i, k + i + 1] = b
    return T


def structure(rng, m, k, kind):
    t = m - k
    theta = np.sort(rng.normal(size=k)) * 3
    s = rng.normal(size=k) * 0.5
    alpha = rng.normal(size=t)
    beta = np.abs(rng.normal(size=max(t - 1, 0))) + 0.1
    if kind == "converged" and k:
        s[rng.random(k) < 0.6] = 0.0          # decoupled pairs arrive with zero coupling
    if kind == "clustered" and k > 8:
        theta[2:6] = theta[2]
        theta[6] = theta[7] * (1 + 1e-15)
    if kind == "tiny":
        beta *= 1e-13
        s *= 1e-12
    if kind == "lanczos":
        alpha = 2 + 0.01 * rng.normal(size=t)
        beta = 1 + 0.01 * np.abs(rng.normal(size=max(t - 1, 0)))
    return theta, s, alpha, beta


CASES = [(1, 0, "plain"), (2, 1, "plain"), (3, 0, "plain"), (40, 0, "plain"), (49, 0, "plain"),
         (97, 0, "lanczos"), (300, 0, "lanczos"), (500, 0, "plain"), (40, 39, "plain"),
         (200, 199, "converged"), (300, 150, "plain"), (300, 250, "converged"),
         (300, 150, "clustered"), (160, 80, "tiny"), (500, 450, "converged"), (1024, 512, "plain")]


@pytest.mark.parametrize("m,k,kind", CASES)
@pytest.mark.parametrize("which", ["lowest", "largest"])
def test_ritz_restart_vs_eigh(ctx, m, k, kind, which):
    from paper_2001_07428_amd import jlanczos as J
    say("ritz_restart", m, k, kind, which)
    rng = np.random.default_rng(1000 * m + k)
    theta, s, alpha, beta = structure(rng, m, k, kind)
    T = assemble(theta, s, alpha, beta)
    lam, Z = J.jl_ritz_restart(ctx, theta, s, alpha, beta, which)
    lam, Z = lam.cpu().numpy(), Z.cpu().numpy()
    ref = np.linalg.eigvalsh(T)
    if which == "largest":
        ref = ref[::-1]
    scale = max(np.abs(T).max(), 1e-300)
    assert np.abs(lam - ref).max() <= 1e-13 * scale * max(1, np.log2(m))
    assert np.abs(Z.T @ Z - np.eye(m)).max() <= 1e-12 * max(1, np.log2(m))
    assert np.abs(T @ Z - Z * lam).max() <= 1e-12 * scale * max(1, np.log2(m))


def test_ritz_restart_matches_jacobi(ctx):
    """The structured solver and the dense Jacobi path agree on the same T."""
    import torch
    from paper_2001_07428_amd import jlanczos as J
    say("ritz_restart vs jacobi")
    rng = np.random.default_rng(5)
    theta, s, alpha, beta = structure(rng, 120, 60, "converged")
    T = assemble(theta, s, alpha, beta)
    l1, Z1 = J.jl_ritz_restart(ctx, theta, s, alpha, beta)
    l2, Z2 = J.jl_ritz(ctx, torch.from_numpy(T).cuda())
    l1, l2 = l1.cpu().numpy(), l2.cpu().numpy()
    assert np.abs(l1 - l2).max() <= 1e-13 * np.abs(T).max()
    # eigenvectors agree up to sign (the spectrum of this T is simple)
    dots = np.abs(np.sum(Z1.cpu().numpy() * Z2.cpu().numpy(), axis=0))
    assert np.abs(dots - 1).max() < 1e-9


def test_ritz_restart_rejects_bad_arguments(ctx):
    from paper_2001_07428_amd import jlanczos as J
    with pytest.raises(ValueError):
        J.jl_ritz_restart(ctx, [1.0], [0.5, 0.1], [1.0], [])
    with pytest.raises(J.JLError):
        J.jl_ritz_restart(ctx, np.zeros(600), np.zeros(600), np.ones(500), np.ones(499))
