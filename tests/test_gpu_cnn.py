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
