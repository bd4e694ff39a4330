"""The allocation-free gradient entry point (wt_mlp_gradient_noalloc) against the allocating one
(wt_mlp_gradient): bitwise equal gradient and loss on two calls in a row, the second with fewer
samples than the first (the shared scratch array keeps the first call's contents)."""
import numpy as np
import pytest

from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (n, 64)).astype(np.float32)
    Y = (rng.random((n, 4)) < 0.35).astype(np.float32)
    return X, Y


def test_gradient_noalloc_equals_the_allocating_entry_point():
    import torch
    rng = np.random.default_rng(17)
    theta = (inputs.mlp_init() + rng.normal(0, 0.02, wt.MLP_PARAMS)).astype(np.float32)
    with wt.Mlp(theta) as m:
        for n in (1000, 37):
            print(f"[no-alloc] n={n}", flush=True)
            X, Y = _data(n, 100 + n)
            x, y = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
            out = torch.full((wt.MLP_PARAMS + 1,), float("nan"), dtype=torch.float32, device="cuda")
            m.gradient_noalloc(x, y, out)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            g, loss = m.gradient(x, y)
            assert np.array_equal(got[:wt.MLP_PARAMS], g)
            assert float(got[wt.MLP_PARAMS]) / (4.0 * n) == loss
            assert np.isfinite(got).all()
        big = torch.zeros((1025, 64), dtype=torch.float32, device="cuda")
        with pytest.raises(wt.WtError):
            m.gradient_noalloc(big, torch.zeros((1025, 4), dtype=torch.float32, device="cuda"), out)
