"""CPU pins of the selector-network reference (oracle/mlp.py) against torch's own
implementations: autograd in float64 for the loss and its gradient, torch.optim.Adam for
the optimiser step, torch's bfloat16 conversion for the rounding rule, and central
finite differences of the loss.  None of these share code with the reference."""
import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, 16)) * 2 + 1
    y = rng.integers(0, 8, B)
    w = rng.standard_normal(omlp.NPARAM) * 0.2
    mu = rng.standard_normal(16) * 0.3
    isd = 0.5 + rng.random(16)
    cw = 0.5 + rng.random(8)
    return X, y, w, mu, isd, cw


class _Net(torch.nn.Module):
    """16 -> 64 -> 64 -> 8 with ReLU, float64, weights taken from the flat vector."""

    def __init__(self, w):
        super().__init__()
        t = torch.as_tensor(np.asarray(w, np.float64))
        self.l1 = torch.nn.Linear(16, 64).double()
        self.l2 = torch.nn.Linear(64, 64).double()
        self.l3 = torch.nn.Linear(64, 8).double()
        with torch.no_grad():  # flat layout: W [in][out] row-major, then bias
            self.l1.weight.copy_(t[0:1024].reshape(16, 64).T)
            self.l1.bias.copy_(t[1024:1088])
            self.l2.weight.copy_(t[1088:5184].reshape(64, 64).T)
            self.l2.bias.copy_(t[5184:5248])
            self.l3.weight.copy_(t[5248:5760].reshape(64, 8).T)
            self.l3.bias.copy_(t[5760:5768])

    def forward(self, xn):
        return self.l3(torch.relu(self.l2(torch.relu(self.l1(xn)))))

    def flat_grad(self):
        return torch.cat([self.l1.weight.grad.T.reshape(-1), self.l1.bias.grad, self.l2.weight.grad.T.reshape(-1),
                          self.l2.bias.grad, self.l3.weight.grad.T.reshape(-1), self.l3.bias.grad]).numpy()


def test_loss_and_gradient_match_torch_autograd_float64():
    X, y, w, mu, isd, cw = _batch(257, 11)
    net = _Net(w)
    xn = (torch.as_tensor(X) - torch.as_tensor(mu)) * torch.as_tensor(isd)
    # class-weighted softmax cross-entropy, mean weighted by the class weights of the labels
    loss = torch.nn.functional.cross_entropy(net(xn), torch.as_tensor(y), weight=torch.as_tensor(cw))
    loss.backward()
    lref, g = omlp.loss_and_grad(w, X, y, cw, mu, isd)
    assert abs(lref - loss.item()) <= 1e-13 * abs(loss.item())
    gt = net.flat_grad()
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-14 * np.abs(gt).max())


def test_forward_matches_torch():
    X, y, w, mu, isd, cw = _batch(100, 12)
    xn = (torch.as_tensor(X) - torch.as_tensor(mu)) * torch.as_tensor(isd)
    Z = _Net(w)(xn).detach().numpy()
    np.testing.assert_allclose(omlp.forward(w, X, mu, isd)[3], Z, rtol=1e-12, atol=1e-13 * np.abs(Z).max())


def test_gradient_matches_central_finite_differences():
    X, y, w, mu, isd, cw = _batch(300, 1)
    _, g = omlp.loss_and_grad(w, X, y, cw, mu, isd)
    rng = np.random.default_rng(2)
    for p in rng.choice(omlp.NPARAM, 24, replace=False):
        h = 1e-6  # small enough not to straddle ReLU kinks in practice
        wp, wm = w.copy(), w.copy()
        wp[p] += h
        wm[p] -= h
        fd = (omlp.loss_and_grad(wp, X, y, cw, mu, isd)[0] - omlp.loss_and_grad(wm, X, y, cw, mu, isd)[0]) / (2 * h)
        assert abs(fd - g[p]) < 1e-8 + 1e-5 * abs(g[p]), (p, fd, g[p])


@pytest.mark.parametrize("wd", [0.0, 1e-2])
def test_adam_matches_torch_optim_adam(wd):
    """Several steps with torch.optim.Adam (its weight_decay adds wd * w to the gradient,
    coupled L2, which is what the library's step does)."""
    rng = np.random.default_rng(3)
    w = rng.standard_normal(omlp.NPARAM)
    p = torch.nn.Parameter(torch.as_tensor(w.copy()))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in range(1, 8):
        g = rng.standard_normal(omlp.NPARAM)
        p.grad = torch.as_tensor(g.copy())
        opt.step()
        w, m, v = omlp.adam(w, g, m, v, step, 1e-3, 0.9, 0.999, 1e-8, wd)
        np.testing.assert_allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-15)
    st = opt.state[p]
    np.testing.assert_allclose(m, st["exp_avg"].numpy(), rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-12, atol=1e-18)


def test_bf16_rounding_matches_torch_bfloat16():
    rng = np.random.default_rng(4)
    # ordinary values over many magnitudes, both signs
    x = (rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000)).astype(np.float32)
    # exact ties: a BF16 value plus half an ulp (even and odd last kept bit), and their negatives
    base = rng.standard_normal(2000).astype(np.float32)
    u = base.view(np.uint32) & np.uint32(0xFFFF0000)
    ties = np.concatenate([u | np.uint32(0x8000), (u | np.uint32(0x18000)) & np.uint32(0xFFFF8000)]).view(np.float32)
    # the largest finite FP32 values round up to infinity; subnormals and zeros
    specials = np.array([3.4e38, -3.4e38, 1e-40, -1e-40, 0.0, -0.0, 1.0, -1.0], np.float32)
    x = np.concatenate([x, ties, specials])
    ref = torch.as_tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = omlp.bf16(x)
    assert np.array_equal(got, ref, equal_nan=False)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_bf16_forward_matches_torch_bf16_rounded_network():
    """Weights, normalised inputs and hidden activations rounded to BF16 by torch, the
    products and sums in float64."""
    X, y, w, mu, isd, cw = _batch(64, 5)
    w32, X32, mu32, isd32 = (a.astype(np.float32) for a in (w, X, mu, isd))

    def r(t):  # round to bfloat16 through FP32, as the activations are stored
        return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    t = torch.as_tensor(w32.astype(np.float64))
    W1, b1 = r(t[0:1024].reshape(16, 64)), t[1024:1088]
    W2, b2 = r(t[1088:5184].reshape(64, 64)), t[5184:5248]
    W3, b3 = r(t[5248:5760].reshape(64, 8)), t[5760:5768]
    xn = r((torch.as_tensor(X32) - torch.as_tensor(mu32)) * torch.as_tensor(isd32))
    h1 = r(torch.relu(xn @ W1 + b1))
    h2 = r(torch.relu(h1 @ W2 + b2))
    Z = (h2 @ W3 + b3).numpy()
    np.testing.assert_allclose(omlp.forward_bf16(w32, X32, mu32, isd32), Z, rtol=1e-12, atol=1e-13 * np.abs(Z).max())
