"""Parity of the child-patch predictor network on the matrix cores against the FP64 oracle:
forward probabilities, gradient, loss, the Adam update, and that training through the C ABI
lowers the loss of a learnable task.  Sizes span several 16-sample tiles, several 4-tile
workgroups and ragged tails."""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_1404_0405_amd import inputs, wt

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-mlp] {msg}", flush=True)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (n, 64)).astype(np.float32)
    Y = (rng.random((n, 4)) < 0.35).astype(np.float32)
    return X, Y


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [1, 16, 17, 100, 1000])
def test_forward_matches_oracle(n):
    import torch
    _say(f"forward n={n}")
    theta = inputs.mlp_init()
    X, _ = _data(n, 5 + n)
    with wt.Mlp(theta) as m:
        x = _cuda(X)
        p = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        m.forward(x, p)
        torch.cuda.synchronize()
        got = p.cpu().numpy().astype(np.float64)
    th = theta.astype(np.float64)
    z_e, _ = omlp.forward(th, X.astype(np.float64), emulate_bf16=True)
    z_x, _ = omlp.forward(th, X.astype(np.float64))
    pe, px = omlp.sigmoid(z_e), omlp.sigmoid(z_x)
    _say(f"max |p - p_bf16emul| {np.abs(got - pe).max():.2e}, max |p - p_fp64| {np.abs(got - px).max():.2e}")
    assert np.abs(got - pe).max() < 2e-3
    assert np.abs(got - px).max() < 3e-2


@pytest.mark.parametrize("n", [16, 100, 777])
def test_gradient_matches_oracle(n):
    _say(f"gradient n={n}")
    rng = np.random.default_rng(9)
    theta = (inputs.mlp_init() + rng.normal(0, 0.02, wt.MLP_PARAMS)).astype(np.float32)
    X, Y = _data(n, 31 + n)
    with wt.Mlp(theta) as m:
        g, loss = m.gradient(_cuda(X), _cuda(Y))
    th = theta.astype(np.float64)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    ge = omlp.grad(th, Xd, Yd, emulate_bf16=True)
    gx = omlp.grad(th, Xd, Yd)
    le = omlp.loss(th, Xd, Yd, emulate_bf16=True)
    rel_e = np.linalg.norm(g - ge) / np.linalg.norm(ge)
    rel_x = np.linalg.norm(g - gx) / np.linalg.norm(gx)
    cos = float(g @ gx / (np.linalg.norm(g) * np.linalg.norm(gx)))
    _say(f"grad rel err vs bf16-emulating oracle {rel_e:.2e}, vs FP64 oracle {rel_x:.2e}, cos {cos:.6f}; "
         f"loss {loss:.6f} vs {le:.6f}")
    assert rel_e < 1e-2
    assert rel_x < 5e-2 and cos > 0.998
    assert loss == pytest.approx(le, rel=1e-4)
    # every block of the parameter vector is covered
    offs = np.cumsum([0] + [int(np.prod(s)) for s in omlp.SHAPES])
    for k in range(6):
        a, b = g[offs[k]:offs[k + 1]], ge[offs[k]:offs[k + 1]]
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12, k


def test_adam_step_matches_oracle():
    _say("adam")
    theta = inputs.mlp_init()
    X, Y = _data(300, 77)
    with wt.Mlp(theta) as m:
        g, _ = m.gradient(_cuda(X), _cuda(Y))
        m.train_step(_cuda(X), _cuda(Y), 1e-3)
        new = m.params()
    th = theta.astype(np.float64)
    want, _, _ = omlp.adam_step(th, g.astype(np.float64), np.zeros_like(th), np.zeros_like(th), 1, 1e-3)
    assert np.allclose(new, want, rtol=1e-6, atol=1e-7)


def test_training_lowers_loss():
    """A learnable task (each output a threshold of one input feature): the loss falls from
    about log 2 well below it, and the trained network classifies most samples."""
    import torch
    _say("training")
    rng = np.random.default_rng(123)
    n = 4096
    X = rng.normal(0.0, 1.0, (n, 64)).astype(np.float32)
    Y = np.stack([X[:, 3] > 0.2, X[:, 10] < -0.5, X[:, 20] + X[:, 21] > 0, X[:, 40] > 1.0], 1).astype(np.float32)
    x, y = _cuda(X), _cuda(Y)
    with wt.Mlp(inputs.mlp_init()) as m:
        l0 = m.gradient(x, y)[1]
        for it in range(300):
            m.train_step(x, y, 3e-3, want_loss=False)
        l1 = m.gradient(x, y)[1]
        p = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        m.forward(x, p)   # asynchronous on the network's stream
        torch.cuda.synchronize()
        acc = float(((p.cpu().numpy() > 0.5) == (Y > 0.5)).mean())
    _say(f"loss {l0:.4f} -> {l1:.4f}, accuracy {acc:.4f}")
    assert l1 < 0.35 * l0
    assert acc > 0.95


def test_bad_arguments():
    with pytest.raises(ValueError):
        wt.Mlp(np.zeros(10, dtype=np.float32))
    with wt.Mlp(inputs.mlp_init()) as m:
        import torch
        x = torch.zeros((4, 63), dtype=torch.float32, device="cuda")
        with pytest.raises(ValueError):
            m.gradient(x, torch.zeros((4, 4), dtype=torch.float32, device="cuda"))
