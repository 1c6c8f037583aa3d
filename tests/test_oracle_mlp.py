"""Pins of the FP64 MLP reference.

* The analytic gradient equals central finite differences of the loss
  (relative error <= 1e-6 on every parameter block);
* 4417 parameters; Xavier-uniform initial weights lie in +-sqrt(6/(fi+fo))
  with mean ~ 0 and variance a^2/3; biases start at zero;
* the first Adam step moves every parameter with non-zero gradient by lr
  against the sign of its gradient (bias-corrected moments: m^/sqrt(v^) = sign);
* training on the exact entropy deficit of small lattices lowers the loss;
* what the network gains over the method without it, at sizes the CPU
  handles: trained on the weights the plain recursion converges to at
  L = 4, 8, 12, its initial ln W at L = 16 and 24 lies within a few units of
  the exact -ln g (up to a constant), where the flat start is off by the whole
  range of ln g; and the first recorded iteration of walkers prepared at the
  learned weights visits every window level, where the flat start's visits
  only the levels near E = 0.  (The sweeps-to-flat comparison itself runs at
  L = 64, 96, 128 on the GPU.)
"""
import math

import numpy as np

import oracle
from oracle import exact
from oracle import mlp


def _data(n=300, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, 2))
    Y = np.sin(2 * X[:, 0]) * 0.3 + 0.2 * X[:, 1] ** 2 - 0.1
    return X, Y


def test_parameter_count_and_init():
    assert mlp.NPARAMS == 4417
    p = mlp.init_params(7)
    q = mlp.unflatten(p)
    for name, (fo, fi) in (("W1", (64, 2)), ("W2", (64, 64)), ("W3", (1, 64))):
        a = math.sqrt(6.0 / (fi + fo))
        w = q[name].reshape(-1)
        assert np.all(np.abs(w) <= a)
        if w.size > 100:
            assert abs(w.mean()) < 4 * a / math.sqrt(3 * w.size)
            assert abs(w.var() / (a * a / 3.0) - 1.0) < 0.15
    for name in ("b1", "b2", "b3"):
        assert np.all(q[name] == 0)
    assert not np.array_equal(p, mlp.init_params(8))


def test_gradient_matches_finite_differences():
    X, Y = _data()
    p = mlp.init_params(3)
    p = p + np.random.default_rng(1).normal(0, 0.05, p.size)  # non-zero biases too
    loss, g = mlp.loss_and_grad(p, X, Y)
    rng = np.random.default_rng(2)
    off = 0
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        idx = off + rng.choice(n, size=min(n, 12), replace=False)
        for i in idx:
            h = 1e-6 * max(1.0, abs(p[i]))
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (mlp.loss_and_grad(pp, X, Y)[0] - mlp.loss_and_grad(pm, X, Y)[0]) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1e-3, np.max(np.abs(g))), (name, i, fd, g[i])
        off += n


def test_first_adam_step_is_sign_times_lr():
    X, Y = _data()
    p0 = mlp.init_params(3)
    _, g = mlp.loss_and_grad(p0, X, Y)
    p1, _ = mlp.train(p0, X, Y, 1, lr=1e-3)
    nz = np.abs(g) > 1e-4  # well above eps = 1e-8, so |step| = lr to 1e-4
    assert nz.sum() > 1000
    assert np.allclose((p0 - p1)[nz], 1e-3 * np.sign(g[nz]), rtol=2e-4, atol=0)


def test_training_on_exact_entropy_lowers_loss():
    lnW = {}
    for L in (8, 12, 16):
        g = exact.exact_g(L)
        K = L * L // 2
        lng = np.array([exact.big_log(v) if v else 0.0 for v in g[:K + 1]])
        lnW[L] = -(lng - lng[K])  # ln W = -ln g, zero at E = 0
    X, Y = mlp.training_set(lnW)
    p, losses = mlp.train(mlp.init_params(5), X, Y, 300, lr=3e-3)
    assert losses[-1] < 0.05 * losses[0]


def test_learned_start_gains_over_flat_start():
    # converged weights of the plain recursion (ln W = -ln g_est of a short
    # production run) at the training sizes
    lnW = {}
    for L, rec_max in ((4, 10), (8, 40), (12, 40)):
        r = oracle.muca_run(L, 512, 19 + L, eq_sweeps=2, rec_sweeps=10, max_iter=2000, prod_sweeps=400,
                            rec_max=rec_max, prep_sweeps=400, rec_rule=1)
        assert r["converged"], L
        w = -np.where(np.isfinite(r["lng"]), r["lng"], 0.0)
        lnW[L] = w - w[-1]
    X, Y = mlp.training_set(lnW)
    p, losses = mlp.train(mlp.init_params(1), X, Y, 3000)
    assert losses[-1] < 1e-3 * losses[0]

    def spread(L, w):
        # max |ln W + ln g - c| over the reachable levels, best constant c
        K = oracle.muca_levels(L)
        g = exact.exact_g(L)
        reach = oracle.muca_flat_levels(L)
        d = np.array([exact.big_log(g[k]) + w[k] for k in range(K) if reach[k]])
        return (d.max() - d.min()) / 2

    for L, bound in ((16, 4.0), (24, 12.0)):
        K = oracle.muca_levels(L)
        learned, flat = spread(L, mlp.predict_lnW(p, L)), spread(L, np.zeros(K))
        assert learned < bound and learned < flat / 20, (L, learned, flat)

    L, W, seed = 16, 256, 201
    K = oracle.muca_levels(L)
    reach = oracle.muca_flat_levels(L)
    coverage = {}
    for arm, w in (("flat", np.zeros(K)), ("learned", mlp.predict_lnW(p, L))):
        spins, E = oracle.muca_start(L, W, seed)
        oracle.muca_prepare(L, spins, E, seed, w, 200)
        oracle.muca_sweeps(L, spins, E, w, seed, 0, 2, False)
        H = oracle.muca_sweeps(L, spins, E, w, seed, 2, 10, True)
        coverage[arm] = float(np.mean(H[reach] > 0))
    assert coverage["learned"] == 1.0 and coverage["flat"] < 0.3, coverage


def test_forward_gradient_and_adam_match_torch_float64():
    """The network, its MSE gradient and full-batch Adam against torch's own
    modules in float64 on the CPU (an independent implementation of the same
    definitions): 2 -> 64 tanh -> 64 tanh -> 1 with weights [out][in]."""
    import torch

    X, Y = _data(n=150, seed=4)
    p0 = mlp.init_params(3) + 0.01 * np.random.default_rng(5).standard_normal(mlp.NPARAMS)
    q = mlp.unflatten(p0)
    net = torch.nn.Sequential(torch.nn.Linear(2, 64), torch.nn.Tanh(), torch.nn.Linear(64, 64), torch.nn.Tanh(),
                              torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4]), (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
            layer.weight.copy_(torch.from_numpy(q[w]))
            layer.bias.copy_(torch.from_numpy(q[b]))
    Xt, Yt = torch.from_numpy(X), torch.from_numpy(Y)
    y, _ = mlp.forward(p0, X)
    assert np.allclose(y, net(Xt)[:, 0].detach().numpy(), rtol=1e-13, atol=1e-14)
    loss_t = torch.mean((net(Xt)[:, 0] - Yt) ** 2)
    loss_t.backward()
    loss, g = mlp.loss_and_grad(p0, X, Y)
    gt = np.concatenate([t.grad.numpy().reshape(-1) for t in (net[0].weight, net[0].bias, net[2].weight,
                                                               net[2].bias, net[4].weight, net[4].bias)])
    assert abs(loss - loss_t.item()) <= 1e-13 * loss_t.item()
    assert np.allclose(g, gt, rtol=1e-10, atol=1e-14 * np.abs(gt).max())
    # five Adam steps (lr, beta1, beta2, eps as the oracle's defaults)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(5):
        opt.zero_grad()
        torch.mean((net(Xt)[:, 0] - Yt) ** 2).backward()
        opt.step()
    p5, _ = mlp.train(p0, X, Y, 5)
    pt = np.concatenate([t.detach().numpy().reshape(-1) for t in (net[0].weight, net[0].bias, net[2].weight,
                                                                   net[2].bias, net[4].weight, net[4].bias)])
    assert np.allclose(p5, pt, rtol=1e-9, atol=1e-12)
