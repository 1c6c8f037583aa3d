"""GPU MLP (forward, backward, Adam in HIP kernels) against the FP64 oracle.

* initial parameters: bit-identical FP32 values;
* gradient of one forward/backward pass: max |g_gpu - g_ref| <= 1e-4 max |g_ref|
  (FP32 arithmetic against FP64), loss to 1e-5 relative;
* training: the GPU loss curve follows the FP64 Adam trajectory (relative
  1e-3 over 300 epochs) and ends far below its start;
* prediction equals the oracle's forward pass of the same parameters to 1e-5.
The data are the exact entropy deficits of small tori, in the form the
multicanonical weights take (y = -ln W / N, ln W(0) = 0).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
from oracle import mlp

pytestmark = pytest.mark.gpu
mcs = pytest.importorskip("paper_1709_04394_amd")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return mcs.Context(0)


@pytest.fixture(scope="module")
def data():
    lnW = {}
    for L in (8, 12, 16, 24):
        g = exact.exact_g(L)
        K = L * L // 2
        lng = np.array([exact.big_log(v) if v else 0.0 for v in g[:K + 1]])
        lnW[L] = -(lng - lng[K])
    X, Y = mlp.training_set(lnW)
    return X, Y


def test_init_bit_identical(ctx):
    p = ctx.mlp_init(11).cpu().numpy()
    ref = mlp.init_params(11).astype(np.float32)
    assert np.array_equal(p, ref)


def test_gradient_vs_fp64(ctx, data):
    X, Y = data
    p64 = mlp.init_params(3) + np.random.default_rng(4).normal(0, 0.05, mlp.NPARAMS)
    p32 = p64.astype(np.float32)
    loss_ref, g_ref = mlp.loss_and_grad(p32.astype(np.float64), X, Y)
    Xd = torch.from_numpy(X.astype(np.float32)).cuda()
    Yd = torch.from_numpy(Y.astype(np.float32)).cuda()
    g, loss = ctx.mlp_grad(torch.from_numpy(p32).cuda(), Xd, Yd)
    g = g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))
    # the data enter in FP32: compare the loss to the same rounding
    loss_ref32 = mlp.loss_and_grad(p32.astype(np.float64), X.astype(np.float32).astype(np.float64),
                                   Y.astype(np.float32).astype(np.float64))[0]
    assert abs(float(loss.cpu()[0]) - loss_ref32) <= 1e-5 * loss_ref32


def test_training_follows_fp64_adam(ctx, data):
    X, Y = data
    X32, Y32 = X.astype(np.float32), Y.astype(np.float32)
    p0 = mlp.init_params(5)
    pd = torch.from_numpy(p0.astype(np.float32)).cuda()
    log = ctx.mlp_train(pd, torch.from_numpy(X32).cuda(), torch.from_numpy(Y32).cuda(), 300, lr=3e-3)
    log = log.cpu().numpy().astype(np.float64)
    p_ref, log_ref = mlp.train(p0, X32.astype(np.float64), Y32.astype(np.float64), 300, lr=3e-3)
    assert np.all(np.abs(log - log_ref) <= 1e-3 * log_ref + 1e-9), np.max(np.abs(log - log_ref) / log_ref)
    assert log[-1] < 0.05 * log[0]
    # prediction with the trained parameters against the FP64 forward pass
    y = ctx.mlp_predict(pd, torch.from_numpy(X32).cuda()).cpu().numpy()
    y_ref, _ = mlp.forward(pd.cpu().numpy().astype(np.float64), X32.astype(np.float64))
    assert np.max(np.abs(y - y_ref)) <= 1e-5


@pytest.mark.parametrize("L", [16, 64, 128])
def test_lnw_init_vs_fp64(ctx, data, L):
    # initial weights at a size outside the training set: -N y from the GPU
    # forward pass against the FP64 forward pass of the same parameters
    X, Y = data
    pd = ctx.mlp_init(2)
    ctx.mlp_train(pd, torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(Y.astype(np.float32)).cuda(),
                  100, lr=3e-3)
    lnW, fb = ctx.mlp_lnw_init(pd, L)
    assert not fb
    ref = mlp.predict_lnW(pd.cpu().numpy().astype(np.float64), L)
    N = L * L
    assert lnW[-1] == 0.0
    assert np.max(np.abs(lnW - ref)) <= 2e-5 * N


def test_lnw_init_falls_back_to_flat(ctx):
    p = ctx.mlp_init(2)
    p[-1] = float("nan")  # b3: every prediction NaN
    lnW, fb = ctx.mlp_lnw_init(p, 32)
    assert fb and np.all(lnW == 0.0)


def test_training_replays_continue_the_epoch_count(ctx, data):
    # 1200 epochs run as two replays of a 500-epoch graph plus a 200-epoch
    # graph: the first 300 losses equal a 300-epoch call bit for bit, and the
    # curve keeps following the FP64 trajectory across the replay boundaries
    X, Y = data
    X32, Y32 = X.astype(np.float32), Y.astype(np.float32)
    p0 = mlp.init_params(5)
    Xd, Yd = torch.from_numpy(X32).cuda(), torch.from_numpy(Y32).cuda()
    pa = torch.from_numpy(p0.astype(np.float32)).cuda()
    pb = torch.from_numpy(p0.astype(np.float32)).cuda()
    short = ctx.mlp_train(pa, Xd, Yd, 300, lr=3e-3).cpu().numpy()
    long_ = ctx.mlp_train(pb, Xd, Yd, 1200, lr=3e-3).cpu().numpy()
    assert np.array_equal(long_[:300], short)
    _, log_ref = mlp.train(p0, X32.astype(np.float64), Y32.astype(np.float64), 700, lr=3e-3)
    rel = np.abs(long_[:700].astype(np.float64) - log_ref) / log_ref
    assert np.max(rel) <= 1e-2, np.max(rel)
    assert np.all(np.isfinite(long_)) and long_[-1] < long_[500] < long_[0]
