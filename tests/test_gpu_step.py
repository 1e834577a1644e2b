"""GPU cross approximation, truncation and full LoMaC-SLAR steps against
the CPU oracle on the same seeded inputs.

Both sides run the same deterministic pivoting rules in FP64, so the pivots
and ranks coincide.  The reconstructed tensors then agree to a tolerance set
by the conditioning of the leaf truncation: the GPU takes leaf bases from
Jacobi eigenvectors of FP64 Gram matrices (the oracle from SVDs of the
unfoldings), and a Gram eigenvector of a kept singular value sigma carries
an error of about eps sigma_1^2 / sigma^2, i.e. eps sigma_1^2 / sigma in the
tensor.  With sigma >= theta = tol ||F|| / sqrt(2d - 3) and at most r kept
directions per leaf this is at most r eps sqrt(2d - 3) / tol of ||F|| per
truncation; fp64_bound() adds it over the truncations of the run.
Conservation is exact up to round-off and checked at 1e-12."""
import numpy as np
import pytest

import slar_inputs as SI
from oracle import ht as HT
from oracle import step as ST

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_29027_amd import lib as L  # noqa: E402
from paper_2606_29027_amd.solver import Solver  # noqa: E402
from gpu_util import normwise  # noqa: E402


def fp64_bound(p, truncations):
    """Gram-conditioning bound of the module docstring (relative, normwise)."""
    return truncations * p.rmax * np.finfo(float).eps * np.sqrt(2 * p.d - 3) / p.tol


def _probes(p):
    Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
    return SI.probe_indices(Nx, Nv, 64, 99)


@pytest.mark.parametrize("name,N,steps", [("landau1d", 32, 3), ("landau2d", 12, 1)])
def test_plain_slar_steps_match_oracle(name, N, steps):
    p = SI.config(name, n=N).with_(lomac=False, alpha=0.2, rmax=40)
    pr = _probes(p)
    o = ST.Oracle(p, probes=pr)
    s = Solver(p, L.F64, probes=pr)
    F0 = SI.initial_ht(p)
    s.set_initial(F0)
    Fo = F0
    o.efield(F0)
    for _ in range(steps):
        Fo = o.strang(Fo, p.dt) if p.split else o.slar_vp(Fo, p.dt)
        s.step()
    assert [st["rank"] for st in s.stats] == [st["rank"] for st in o.stats]
    err = normwise(s.dense(), HT.full(Fo))
    assert err < fp64_bound(p, 3 * steps), err   # conditioning bound, see module docstring


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_lomac_steps_match_oracle_and_conserve(prec):
    """Both Newton solves are driven to 1e-13 so that the two macroscopic
    states agree to round-off, not only to the Newton tolerance."""
    p = SI.config("landau2d", n=12).with_(alpha=0.2, rmax=40)
    pr = _probes(p)
    o = ST.Oracle(p, probes=pr, newton_tol=1e-13)
    s = Solver(p, prec, probes=pr, newton_tol=1e-13)
    F0 = SI.initial_ht(p)
    s.set_initial(F0)
    d0 = s.diagnostics()
    Fo, _ = o.run(F0, 2)
    for _ in range(2):
        info = s.step()
        assert info["converged"]
    d = s.diagnostics()
    assert abs(d["mass"] - d0["mass"]) < 1e-12 * d0["mass"]
    assert abs(d["energy"] - d0["energy"]) < 1e-12 * d0["energy"]
    assert max(abs(m) for m in d["momentum"]) < 1e-12 * d0["mass"]
    err = normwise(s.dense(), HT.full(Fo))
    assert err < (fp64_bound(p, 6) if prec == L.F64 else 10 * p.tol), err


def test_spectral_preconditioner_same_root_fewer_iterations():
    """Preconditioning changes only the Krylov path: the Newton root agrees
    with the unpreconditioned one to the Newton tolerance, in fewer Krylov
    iterations, and conservation is unchanged."""
    p = SI.config("stronglandau2d", n=16).with_(rmax=40)
    pr = _probes(p)
    out = {}
    for pc in (0, 1):
        s = Solver(p, L.F64, probes=pr, precond=pc, newton_tol=1e-12)
        s.set_initial(SI.initial_ht(p))
        d0 = s.diagnostics()
        infos = [s.step() for _ in range(2)]
        d = s.diagnostics()
        assert abs(d["mass"] - d0["mass"]) < 1e-12 * d0["mass"]
        assert abs(d["energy"] - d0["energy"]) < 1e-12 * d0["energy"]
        out[pc] = (s.U_n.cpu().numpy(), sum(i["krylov"] for i in infos))
    assert normwise(out[1][0], out[0][0]) < 1e-9
    assert out[1][1] < out[0][1], (out[0][1], out[1][1])
