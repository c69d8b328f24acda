"""The allocation-free network gradient (gdw_mlp_grad_noalloc, include/gdw.h) against the
allocating one (gdw_mlp_grad) through the C ABI: two calls in a row on the same network,
the second with fewer rows, so the shared scratch array holds the first call's larger
contents when the second runs.  Both run the same kernels in the same order, so the
gradients and losses agree to FP32 rounding (bar 1e-6 relative, l2 and max); the
requests beyond the scratch limit are refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NI, H, K = 64, 128, 168


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_noalloc_gradient_equals_allocating_one():
    import torch
    from _cmp import assert_close
    from paper_2105_01722_amd import gdw
    _say("case: mlp gradient without allocation, n = 300 then 77")
    net = gdw.Mlp(NI, H, K, seed=3, max_batch=512)
    rng = np.random.default_rng(4)
    try:
        for n in (300, 77):
            x = torch.from_numpy(rng.standard_normal((n, NI)).astype(np.float32)).cuda()
            y = torch.from_numpy((0.1 * rng.standard_normal((n, K))).astype(np.float32)).cuda()
            g_ref, l_ref = net.grad(x, y)
            g = torch.full((net.np,), float("nan"), dtype=torch.float32, device="cuda")
            loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
            net.grad_noalloc(x, y, g, loss)
            torch.cuda.synchronize()
            gh, gr = g.cpu().numpy(), g_ref.cpu().numpy()
            _say("  n = %d: max |diff| grad %.2e, loss %.6e vs %.6e"
                 % (n, np.abs(gh - gr).max(), loss.item(), l_ref))
            assert np.isfinite(gh).all()
            assert_close(gh, gr, 1e-6, max_bar=1e-6)
            assert abs(loss.item() - l_ref) <= 1e-6 * abs(l_ref)
        # beyond the 8 MiB scratch: refused before any launch
        n_big = 4000
        x = torch.zeros((n_big, NI), dtype=torch.float32, device="cuda")
        y = torch.zeros((n_big, K), dtype=torch.float32, device="cuda")
        with pytest.raises(gdw.GdwError) as ei:
            net.grad_noalloc(x, y, torch.empty(net.np, dtype=torch.float32, device="cuda"),
                             torch.empty(1, dtype=torch.float64, device="cuda"))
        assert ei.value.status == gdw.GDW_EINVAL
    finally:
        net.close()
