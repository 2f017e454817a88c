"""The allocation-free reorthogonalisation pass (static device scratch)
against the workspace form of the same pass, through the C ABI: three calls in
a row on one context, each later one with a shorter vector, each bit-identical to
jl_reorth_pass (same kernels, same launch shapes, same summation order)."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_pass_matches_workspace_pass(mixed):
    import torch
    from paper_2001_07428_amd import jlanczos as J
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dt = torch.complex64 if mixed else torch.complex128
    ctx = J.Context(0)
    g = torch.Generator(device="cuda:0").manual_seed(11)
    coef = torch.full((4 * 256 + 2,), np.nan, dtype=torch.float64, device="cuda:0")
    # a long vector (the FP32 inner products and update then keep u and the
    # corrections in LDS; a last block of two pairs), a pass at the largest
    # basis width the scratch takes, then a smaller one
    for n, ncol in ((2 * (2097152 + 2), 3), (2 * 262144, 256), (2 * 1531, 37)):
        say("noalloc pass", "mixed" if mixed else "fp64", n, ncol)
        V = torch.randn((ncol, n), dtype=dt, device="cuda:0", generator=g)
        V /= torch.linalg.vector_norm(V, dim=1, keepdim=True)
        u0 = torch.randn(n, dtype=dt, device="cuda:0", generator=g)
        u_ws = u0.clone()
        c_ws = J.jl_reorth_pass(ctx, V, u_ws)
        u_na = u0.clone()
        coef.fill_(np.nan)
        J.jl_reorth_pass_noalloc(ctx, V, u_na, coef)
        torch.cuda.synchronize()
        k = 4 * ncol + 2
        assert torch.equal(coef[:k], c_ws), (n, ncol)
        assert torch.equal(u_na, u_ws), (n, ncol)
        assert torch.isnan(coef[k:]).all()          # nothing written past 4*ncol + 2
    with pytest.raises(J.JLError) as e:              # beyond the scratch: a clear error
        Vb = torch.zeros((257, 64), dtype=dt, device="cuda:0")
        J.jl_reorth_pass_noalloc(ctx, Vb, torch.zeros(64, dtype=dt, device="cuda:0"),
                                 torch.zeros(4 * 257 + 2, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == J.JL_EINVAL
    # the longest vector the scratch takes (norm only), then the next longer
    # one that the long-vector inner products take: a clear error (FP32 with
    # an even half length up to 16777216 elements, FP64 up to 8388608)
    nmax = 16777216 if mixed else 8388608
    u0 = torch.randn(nmax, dtype=dt, device="cuda:0", generator=g)
    c_ws = J.jl_reorth_pass(ctx, None, u0.clone())
    coef.fill_(np.nan)
    J.jl_reorth_pass_noalloc(ctx, None, u0.clone(), coef)
    torch.cuda.synchronize()
    assert torch.equal(coef[:2], c_ws)
    del u0
    with pytest.raises(J.JLError) as e:
        J.jl_reorth_pass_noalloc(ctx, None, torch.zeros(nmax + (4 if mixed else 2), dtype=dt,
                                                         device="cuda:0"), coef)
    assert e.value.status == J.JL_EINVAL
