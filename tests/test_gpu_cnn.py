"""Learned preconditioner: GPU forward/backward against the CPU oracle,
training on solver-generated Newton systems, and the same Newton root with
fewer Krylov iterations than plain GMRES."""
import numpy as np
import pytest

import slar_inputs as SI
from oracle import cnn as CN

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_29027_amd import lib as L  # noqa: E402
from paper_2606_29027_amd import cnn as CNN  # noqa: E402
from paper_2606_29027_amd.solver import Solver  # noqa: E402
from gpu_util import normwise  # noqa: E402


def _net(chs, seed):
    net = L.Cnn(chs, 4, 24 * 20)
    rng = np.random.default_rng(seed)
    theta = (0.3 * rng.standard_normal(net.nparams)).astype(np.float32)
    net.set_params(theta)
    return net, theta.astype(np.float64)


@pytest.mark.parametrize("H,W", [(8, 8), (24, 20)])
def test_cnn_forward_and_gradient_match_oracle(H, W):
    chs = [8, 16, 16, 4]
    net, theta = _net(chs, 3)
    shapes = list(zip(chs[:-1], chs[1:]))
    rng = np.random.default_rng(4)
    x = rng.standard_normal((3, 8, H, W)).astype(np.float32)
    y = rng.standard_normal((3, 4, H, W)).astype(np.float32)
    xd = torch.as_tensor(x, device="cuda"); yd = torch.as_tensor(y, device="cuda")
    out = torch.zeros((3, 4, H, W), dtype=torch.float32, device="cuda")
    net.forward(xd, out)
    ref, _ = CN.forward(theta, shapes, x.astype(np.float64))
    assert normwise(out.cpu().numpy(), ref) < 1e-5
    g, loss = net.grad(xd, yd)
    gref = CN.grad(theta, shapes, x.astype(np.float64), y.astype(np.float64))
    assert abs(loss - CN.loss(theta, shapes, x, y)) < 1e-5 * abs(loss)
    assert normwise(g, gref) < 1e-4


def test_training_reduces_loss_on_recorded_systems():
    p = SI.config("landau2d", n=16).with_(rmax=30)
    data = CNN.collect([p], steps=3, capacity=24)
    assert data[0][0].shape[0] > 4
    net = CNN.make(max_batch=8, max_pixels=16 * 16)
    hist = CNN.train(net, data, iters=60, batch=8, lr=3e-3)
    assert np.mean(hist[-10:]) < np.mean(hist[:3])


def test_learned_preconditioner_same_root_fewer_iterations_than_plain():
    p = SI.config("stronglandau2d", n=16).with_(rmax=40)
    data = CNN.collect([SI.config("landau2d", n=16).with_(rmax=30)], steps=3, capacity=24)
    net = CNN.make(max_batch=8, max_pixels=16 * 16)
    CNN.train(net, data, iters=40, batch=8)
    Nx = 256
    pr = SI.probe_indices(Nx, Nx, 64, 5)
    out = {}
    for pc, cnn in ((0, None), (2, net)):
        s = Solver(p, L.F64, probes=pr, precond=pc, cnn=cnn, newton_tol=1e-12)
        s.set_initial(SI.initial_ht(p))
        d0 = s.diagnostics()
        infos = [s.step() for _ in range(2)]
        d = s.diagnostics()
        assert abs(d["mass"] - d0["mass"]) < 1e-12 * d0["mass"]
        out[pc] = (s.U_n.cpu().numpy(), sum(i["krylov"] for i in infos))
    assert normwise(out[2][0], out[0][0]) < 1e-9
    assert out[2][1] < out[0][1]


def test_recorded_features_are_standardised():
    """Every recorded network input has the normalisation of oracle.cnn.features:
    U channels of mean 0 and std 1 one by one, residual channels of rms 1
    over all channels together (FP32 inputs: bar 1e-5)."""
    p = SI.config("stronglandau2d", n=16).with_(rmax=40)
    K = p.dv + 2
    feats, targs, _ = CNN.collect([p], steps=2, capacity=16)[0]
    f = feats.double().cpu().numpy()
    assert f.shape[0] > 4 and np.all(np.isfinite(f)) and np.all(np.isfinite(targs.cpu().numpy()))
    for q in range(f.shape[0]):
        assert abs(np.sqrt(np.mean(f[q, :K] ** 2)) - 1.0) < 1e-5, q
        for c in range(K):
            u = f[q, K + c]
            assert abs(u.mean()) < 1e-5, (q, c)
            assert abs(u.std() - 1.0) < 1e-5, (q, c)


def test_learned_solve_is_bitwise_reproducible():
    """Two learned-preconditioner runs from the same state give the same bits
    (no atomics, fixed reduction orders), with a network whose output
    depends on every normalisation statistic."""
    p = SI.config("stronglandau2d", n=16).with_(rmax=40)
    chs = CNN.channels(p.dv)
    net = L.Cnn(chs, 8, 16 * 16)
    rng = np.random.default_rng(21)
    net.set_params((0.05 * rng.standard_normal(net.nparams)).astype(np.float32))
    pr = SI.probe_indices(256, 256, 64, 5)
    runs = []
    for _ in range(2):
        s = Solver(p, L.F64, probes=pr, precond=2, cnn=net)
        s.set_initial(SI.initial_ht(p))
        infos = [s.step() for _ in range(2)]
        X, P = s.frames_buf[s.state_slot]
        r = s.state.r
        runs.append((s.U_n.cpu().numpy(), X[:, :r].cpu().numpy(), P[:, :r].cpu().numpy(),
                     [(i["newton"], i["krylov"]) for i in infos]))
    (U0, X0, P0, it0), (U1, X1, P1, it1) = runs
    assert it0 == it1
    assert np.array_equal(U0, U1) and np.array_equal(X0, X1) and np.array_equal(P0, P1)
