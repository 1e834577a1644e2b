"""The allocation-free Poisson entry point against slar_poisson, through
the C ABI: two calls in a row on the same device scratch array, the second
on a smaller grid (and a non-power-of-two one, the direct-DFT lines), then
a third on the first grid again; each matches the workspace entry point to
1e-12 (FP64 normwise) in phi and E."""
import math

import numpy as np
import pytest

import slar_inputs as SI

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_29027_amd import lib as L  # noqa: E402
from gpu_util import dev, normwise  # noqa: E402


def _case(shape, seed):
    dx = len(shape)
    lengths = [4 * math.pi, 3.0][:dx]
    p = SI.Problem("t", dx, dx, tuple(shape) * 2, tuple([0.0] * dx + [-6.0] * dx),
                   tuple(lengths + [6.0] * dx), "landau", 0.1, 0.5)
    g = L.make_grid(p)
    Nx = int(np.prod(shape))
    ne = dev((1.0 + 0.3 * SI.random_field(shape, seed, smooth=False)).ravel())
    return g, Nx, dx, ne


def _both(shape, seed):
    g, Nx, dx, ne = _case(shape, seed)
    ws = L.Workspace(g, 8)
    phi_a = torch.zeros(Nx, dtype=torch.float64, device="cuda")
    E_a = torch.zeros((dx, Nx), dtype=torch.float64, device="cuda")
    L.slar_poisson(g, ne, 1.0, phi_a, E_a, ws)
    phi_b = torch.full((Nx,), float("nan"), dtype=torch.float64, device="cuda")
    E_b = torch.full((dx, Nx), float("nan"), dtype=torch.float64, device="cuda")
    L.slar_poisson_noalloc(g, ne, 1.0, phi_b, E_b)
    torch.cuda.synchronize()
    return (phi_a.cpu().numpy(), E_a.cpu().numpy()), (phi_b.cpu().numpy(), E_b.cpu().numpy())


def test_noalloc_poisson_matches_workspace_entry_point():
    for shape, seed in (((128, 128), 3), ((24, 40), 4), ((128, 128), 5), ((64,), 6)):
        (pa, Ea), (pb, Eb) = _both(shape, seed)
        assert np.all(np.isfinite(pb)) and np.all(np.isfinite(Eb))
        assert normwise(pb, pa) < 1e-12, shape
        assert normwise(Eb, Ea) < 1e-12, shape


def test_noalloc_poisson_rejects_bad_arguments():
    g, Nx, dx, ne = _case((16, 16), 1)
    E = torch.zeros((dx, Nx), dtype=torch.float64, device="cuda")
    with pytest.raises(L.SlarError):
        L.slar_poisson_noalloc(g, ne, float("nan"), None, E)
    bad = L.make_grid(SI.config("stronglandau2d", n=8))
    bad.n[0] = 256                      # beyond the 2D grid limit
    with pytest.raises(L.SlarError):
        L.slar_poisson_noalloc(bad, ne, 1.0, None, E)
