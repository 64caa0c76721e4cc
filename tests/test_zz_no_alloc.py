"""GPU test of the allocation-free null-space projection against the allocating entry point:
two calls in a row on the same device (the second on a smaller grid, so the fixed scratch holds
the larger call's data when it starts), FP64 and FP32, 2D and 3D; bit-identical results (the
same kernels and summation order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_project_null_noalloc_matches_allocating_entry(pd, prec):
    import torch
    dt = torch.float32 if prec == 1 else torch.float64
    cases = [(3, (9, 7, 5), 5), (2, (6, 5), 3), (3, (4, 3, 3), 8), (2, (3, 2), 1)]
    for dim, cells, N in cases:
        print(f"noalloc projection prec={prec} dim={dim} cells={cells} N={N}", flush=True)
        ctx = pd.pd_setup(dim, cells, (1.0,) * dim, N, 1e-3, 0.6, 1e-3)
        rng = np.random.default_rng(N + 10 * dim)
        v0 = torch.tensor(rng.standard_normal(ctx.ndof), dtype=dt, device="cuda")
        a = v0.clone()
        b = v0.clone()
        pd.pd_project_null(ctx, prec, a)
        pd.pd_project_null_noalloc(ctx, prec, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert float((a.double() - v0.double()).abs().max()) > 0.0   # the projection acted
        ctx.close()
