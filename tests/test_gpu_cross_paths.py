"""The stopping paths of the GPU cross approximation against the oracle's
(section 3.1, the adaptive cross with partial pivoting and the random-probe
check that the oracle's `aca` spells out step by step).

The frame tables are given directly and the update is a zero time step, so
the sampled matrix is exactly A = X P^T and the oracle samples that product.
A 12^4 grid gives 144 x 144 (three fiber tiles of 64 entries, the last one
ragged), and 256 probe entries are spread over several column blocks.

Cases: an all-zero tensor (the first row is already reproduced: no term),
an exact rank-3 tensor (the fourth row is reproduced: probe check, then
stop), a rank-2 smooth part plus one entry that the pivots never visit
(the norm test stops, a probe finds the entry, the cross resumes at its
row), the same without probes, and the term cap reached before the norm
test stops; and seeded random cases across them."""
import numpy as np
import pytest

import slar_inputs as SI
from oracle import cross as CR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2606_29027_amd import lib as L  # noqa: E402

N = 12
NX = N * N


def _probes(count, seed, extra=None):
    pr = SI.probe_indices(NX, NX, count, seed)
    if extra is not None:
        pr = np.array(pr, copy=True)
        pr[150] = extra            # in the probe share of the third column block
    return pr


def _cross(X, P, tol, kmax, probes):
    """GPU cross (FP64 tables) and the oracle's on A = X P^T."""
    r = X.shape[1]
    p = SI.config("stronglandau2d", n=N).with_(tol=tol)
    g = L.make_grid(p)
    ws = L.Workspace(g, 64)
    Xd = torch.zeros(NX, 72, dtype=torch.float64, device="cuda")
    Pd = torch.zeros(NX, 72, dtype=torch.float64, device="cuda")
    Xd[:, :r] = torch.as_tensor(X)
    Pd[:, :r] = torch.as_tensor(P)
    src = L.frames(Xd, Pd, r)
    adv = L.make_adv(0, 0.0, 1.0)
    U = torch.zeros(kmax, NX, dtype=torch.float64, device="cuda")
    V = torch.zeros(kmax, NX, dtype=torch.float64, device="cuda")
    pr = None if probes is None else torch.as_tensor(probes, dtype=torch.int32, device="cuda")
    lr, info, st = L.slar_cross_update(g, src, adv, L.F64, tol, kmax, pr, U, V, ws)
    torch.cuda.synchronize()
    A = X @ P.T
    Uo, Vo, io = CR.aca(lambda i: A[i], lambda j: A[:, j], lambda I, J: A[I, J], NX, NX, tol, kmax, 0,
                        probes)
    k = info.rank
    got = U[:k].cpu().numpy().T @ V[:k].cpu().numpy() if k > 0 else np.zeros_like(A)
    return dict(info=info, st=st, got=got, A=A, Uo=Uo, Vo=Vo, io=io, k=k)


def _smooth(seed, r):
    rng = np.random.default_rng(seed)
    t = np.linspace(0.0, 2.0 * np.pi, NX, endpoint=False)
    X = np.stack([np.cos((m + 1) * t + rng.uniform(0, 6)) + 0.3 * rng.standard_normal() for m in range(r)], 1)
    P = np.stack([np.exp(-((t - rng.uniform(1, 5)) ** 2)) * (m + 1.0) for m in range(r)], 1)
    return X, P


def test_zero_tensor_stops_without_terms():
    X = np.zeros((NX, 2))
    P = np.zeros((NX, 2))
    c = _cross(X, P, 1e-6, 16, _probes(256, 3))
    assert c["st"] == L.SLAR_OK
    assert c["k"] == 0 and c["info"].converged == 1 and c["info"].probe_rounds == 0
    assert c["info"].samples == NX              # one row, no probes (nothing to check against)
    assert c["io"]["converged"] and not c["io"]["pivots"]


@pytest.mark.parametrize("with_probes", [True, False])
def test_exact_rank_three_stops_at_the_reproduced_row(with_probes):
    rng = np.random.default_rng(11)
    X = rng.standard_normal((NX, 3))
    P = rng.standard_normal((NX, 3))
    probes = _probes(256, 5) if with_probes else None
    c = _cross(X, P, 1e-6, 32, probes)
    io = c["io"]
    assert c["st"] == L.SLAR_OK and c["info"].converged == 1
    assert io["converged"] and io["rank"] == 3 and io["probe_rounds"] == 0
    assert c["k"] == 3 and c["info"].probe_rounds == 0
    # rows of the three terms, the reproduced fourth row, then the probes
    assert c["info"].samples == io["samples"]
    scale = np.abs(c["A"]).max()
    assert np.abs(c["got"] - c["Uo"] @ c["Vo"].T).max() < 1e-12 * scale
    assert np.abs(c["got"] - c["A"]).max() < 1e-12 * scale


def test_probe_finds_an_entry_the_pivots_missed():
    X, P = _smooth(21, 2)
    x0, v0 = 97, 130
    A = X @ P.T
    spike = 1e-3 * np.abs(A).max()
    X = np.concatenate([X, spike * np.eye(NX, 1, -x0)], 1)
    P = np.concatenate([P, np.eye(NX, 1, -v0)], 1)
    c = _cross(X, P, 1e-6, 32, _probes(256, 9, extra=(x0, v0)))
    io = c["io"]
    # the input does what the case is about (oracle): one probe round that
    # restarts at the spike's row, then convergence
    assert io["probe_rounds"] == 1 and io["converged"], io
    assert (x0, v0) in [tuple(pv) for pv in io["pivots"]]
    assert c["st"] == L.SLAR_OK and c["info"].converged == 1
    assert c["k"] == io["rank"] and c["info"].probe_rounds == 1
    assert c["info"].samples == io["samples"]
    scale = np.abs(c["A"]).max()
    assert np.abs(c["got"] - c["Uo"] @ c["Vo"].T).max() < 1e-12 * scale
    assert abs(c["got"][x0, v0] - c["A"][x0, v0]) < 1e-12 * scale


def test_term_cap_before_the_norm_test_stops():
    rng = np.random.default_rng(17)
    X = rng.standard_normal((NX, 3))
    P = rng.standard_normal((NX, 3))
    c = _cross(X, P, 1e-6, 2, _probes(256, 5))
    io = c["io"]
    assert not io["converged"] and io["rank"] == 2
    assert c["st"] == L.SLAR_E_RANK_CAP and c["k"] == 2 and c["info"].converged == 0
    assert c["info"].samples == io["samples"]
    scale = np.abs(c["A"]).max()
    assert np.abs(c["got"] - c["Uo"] @ c["Vo"].T).max() < 1e-12 * scale


@pytest.mark.parametrize("seed", range(16))
def test_random_low_rank_cases_match_the_oracle(seed):
    """Seeded random cases over the same paths: rank 1..6 with a decaying
    spectrum, sometimes one entry the pivots miss (inside the probe set),
    0, 64 or 300 probes, tolerance 1e-4 or 1e-8, term cap 2, 4 or 32 (at
    the cap the last term is far above the tolerance, so both sides stop
    as capped).  Rank, stopping flags, probe rounds, sample counts and
    U V^T agree with the oracle."""
    rng = np.random.default_rng(1000 + seed)
    r = int(rng.integers(1, 7))
    X = rng.standard_normal((NX, r)) * (0.3 ** np.arange(r))[None, :]
    P = rng.standard_normal((NX, r))
    spike = bool(rng.integers(0, 2))
    if spike:
        x0, v0 = int(rng.integers(0, NX)), int(rng.integers(0, NX))
        X = np.concatenate([X, 1e-3 * np.eye(NX, 1, -x0)], 1)
        P = np.concatenate([P, np.eye(NX, 1, -v0)], 1)
    nprobe = int(rng.choice([0, 64, 300]))
    probes = SI.probe_indices(NX, NX, nprobe, 50 + seed) if nprobe else None
    if spike and nprobe:
        probes = np.array(probes, copy=True)
        probes[nprobe // 2] = (x0, v0)
    tol = float(rng.choice([1e-4, 1e-8]))
    kmax = int(rng.choice([2, 4, 32]))
    c = _cross(X, P, tol, kmax, probes)
    io = c["io"]
    assert c["k"] == io["rank"]
    assert bool(c["info"].converged) == bool(io["converged"])
    assert c["info"].probe_rounds == io["probe_rounds"]
    assert c["info"].samples == io["samples"]
    assert c["st"] == (L.SLAR_OK if io["converged"] else L.SLAR_E_RANK_CAP)
    scale = np.abs(c["A"]).max()
    assert np.abs(c["got"] - c["Uo"] @ c["Vo"].T).max() < 1e-12 * scale
