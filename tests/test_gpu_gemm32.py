"""The restart GEMM V_k = V_m Z (Alg. 1, the thick-restart basis update) at the
32^4 shape: n = 8388608 complex elements per basis vector and m = 500 vectors,
so 16.8M real rows and element offsets of the basis past 2^31.  Sampled entries
of the result are compared with an FP64 NumPy product of the same sampled
entries of the basis (both ends of each half and random ones); k = 300 runs the
columns as 128-wide tiles plus a 64-wide tile, k = 280 plus a 32-wide tile.
Z has orthonormal columns, like the Ritz vectors of the restart."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

N32 = 2 * 32 ** 4 * 4
M32 = 500


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return J.Context(0)


@pytest.mark.parametrize("k,mixed", [(300, True), (280, True), (300, False)])
def test_basis_update_32_4_sampled(ctx, k, mixed):
    import torch
    from paper_2001_07428_amd import jlanczos as J
    say("basis_update 32^4", k, "mixed" if mixed else "fp64")
    dt = torch.complex64 if mixed else torch.complex128
    g = torch.Generator(device="cuda:0").manual_seed(21 + k)
    V = torch.randn((M32, N32), dtype=dt, device="cuda:0", generator=g)
    rng = np.random.default_rng(k)
    Z = np.linalg.qr(rng.standard_normal((M32, k)))[0]
    Y = J.jl_basis_update(ctx, V, torch.from_numpy(Z).cuda())
    torch.cuda.synchronize()
    h = N32 // 2
    idx = np.unique(np.concatenate([[0, 1, h - 1, h, N32 - 2, N32 - 1], rng.integers(0, N32, 250)]))
    it = torch.from_numpy(idx).cuda()
    Vs = V[:, it].cpu().numpy().astype(np.complex128)   # (m, samples), the stored values
    Ys = Y[:, it].cpu().numpy().astype(np.complex128)   # (k, samples)
    del V, Y
    torch.cuda.empty_cache()
    ref = Z.T @ Vs
    # per entry against |Z|^T |V|: one rounding to FP32 (mixed), or the FP64
    # accumulation over m terms (m u_64 = 5.6e-14, doubled)
    err = np.abs(Ys - ref) / (np.abs(Z).T @ np.abs(Vs))
    print(f"  max error {err.max():.2e} over {len(idx)} sampled elements x {k} columns", flush=True)
    assert err.max() < (1e-7 if mixed else 1.2e-13)
