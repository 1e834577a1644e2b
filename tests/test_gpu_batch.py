"""Batched multi-instance path (slar_batch_*): the persistent multi-instance
cross approximation replayed from a captured hipGraph, the grouped skeleton
cores of capped crosses and the grouped truncation against the one-instance
library calls, and whole batched steps against the CPU oracle.

With the default team width (16 lanes per sample) a batched tile runs the
same arithmetic as the one-instance kernels on the same FP32 tables, so U,
V, ranks and iteration counts must agree bit for bit.  Several calls in a
row (three sub-flows, with eager field solves between them) replay the
captured graph; every replay is checked against the eager one-instance call.
Against the FP64 oracle the FP32 tables allow 10 tol (normwise) per step,
the bound the one-instance FP32 step tests use."""
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
from paper_2606_29027_amd.batch import BatchSolver  # noqa: E402
from gpu_util import normwise  # noqa: E402


def _probes(p, seed):
    Nx = int(np.prod(p.n[: p.dx])); Nv = int(np.prod(p.n[p.dx:]))
    return SI.probe_indices(Nx, Nv, 64, seed)


def _solver(problems):
    pr = [_probes(p, 100 + q) for q, p in enumerate(problems)]
    b = BatchSolver(problems, probes=pr)
    b.set_initial([SI.initial_ht(p) for p in problems])
    return b, pr


def _single_cross(b, q, src, adv):
    I = b.inst[q]
    ws = b.batch.ws[q]
    U = torch.zeros_like(I.U); V = torch.zeros_like(I.V)
    lr, info, _ = L.slar_cross_update(ws.grid, src, adv, L.F32, b.tol, b.rmax, b.probes[q], U, V, ws)
    torch.cuda.synchronize()
    return U, V, info


def test_batch_cross_bitwise_equals_single_instance_over_replays():
    problems = SI.batched_instances(10)
    b, _ = _solver(problems)
    assert b.batch.config()["team_r16"] == 16
    h = b.dt
    E1 = b.efield(b.state, 0)
    stages = [(b.state, [L.make_adv(2, h / 3.0, 1.0, E) for E in E1]),
              (b.state, [L.make_adv(2, 2.0 * h / 3.0, 1.0, E) for E in E1]),
              (b.state, [L.make_adv(2, h, 2.0 / 3.0, E, E, (-1.0 / 12.0, 3.0 / 4.0)) for E in E1])]
    for src, advs in stages:
        lrs, info, _ = b.batch.cross_update(src, advs, b.tol, b.rmax, b.probes,
                                            [I.U for I in b.inst], [I.V for I in b.inst])
        torch.cuda.synchronize()
        got = [(I.U.clone(), I.V.clone()) for I in b.inst]
        b.efield(src, 1)                    # eager work between graph replays
        for q in range(b.count):
            U, V, inf = _single_cross(b, q, src[q], advs[q])
            k = inf.rank
            assert info[q].rank == k and info[q].iterations == inf.iterations, q
            assert info[q].samples == inf.samples and info[q].probe_rounds == inf.probe_rounds, q
            assert torch.equal(got[q][0][:k], U[:k]) and torch.equal(got[q][1][:k], V[:k]), q
    assert b.batch.config()["captures"] == 1


def test_batch_capped_crosses_equal_single_instance():
    """Crosses that stop at the term cap (k = 2 rmax > rmax) are replaced by
    the regularised skeleton C W_r^+ R; the batched call groups the pivot-
    block SVDs of all capped instances into one launch per size class.
    Every instance must still get, bit for bit, the terms and rank of the
    one-instance slar_cross_update on a workspace of the same rank cap."""
    problems = SI.batched_instances(10)
    pr = [_probes(p, 100 + q) for q, p in enumerate(problems)]
    b = BatchSolver(problems, probes=pr, rmax=6)
    b.set_initial([SI.initial_ht(p) for p in problems])
    assert b.kcross == 12
    E1 = b.efield(b.state, 0)
    advs = [L.make_adv(2, b.dt / 3.0, 1.0, E) for E in E1]
    lrs, info, _ = b.batch.cross_update(b.state, advs, b.tol, b.kcross, b.probes,
                                        [I.U for I in b.inst], [I.V for I in b.inst])
    torch.cuda.synchronize()
    got = [(I.U.clone(), I.V.clone()) for I in b.inst]
    capped = 0
    for q in range(b.count):
        I = b.inst[q]
        ws = b.batch.ws[q]
        U = torch.zeros_like(I.U); V = torch.zeros_like(I.V)
        lr, inf, st = L.slar_cross_update(ws.grid, b.state[q], advs[q], L.F32, b.tol, b.kcross, b.probes[q],
                                          U, V, ws)
        torch.cuda.synchronize()
        k = inf.rank
        if st == L.SLAR_E_RANK_CAP:         # skeleton of at most rmax terms
            capped += 1
            assert k <= b.rmax, q
        assert info[q].rank == k, q
        assert torch.equal(got[q][0][:k], U[:k]) and torch.equal(got[q][1][:k], V[:k]), q
    assert capped >= 2


def test_batch_efield_equals_single_instance():
    """The batched field solve runs the moments (chunked products and their
    fixed-order sum) and the spectral Poisson solve (line FFTs for powers of
    two, DFTs for N = 48 and 96) as one grouped launch per step over all
    instances: moments and field must equal, bit for bit, those of the
    one-instance slar_moments and slar_poisson.  Two calls in a row without
    a synchronisation between them share the staging memory."""
    problems = SI.batched_instances(12)
    assert {p.n[0] for p in problems} & {48, 96}
    b, _ = _solver(problems)
    E0 = [e.clone() for e in b.efield(b.state, 0)]
    b.efield(b.state, 1)
    torch.cuda.synchronize()
    for q, p in enumerate(problems):
        I = b.inst[q]
        ws = b.batch.ws[q]
        M = torch.zeros_like(I.M)
        E = torch.zeros_like(I.E[0])
        L.slar_moments(ws.grid, b.state[q], M, ws)
        L.slar_poisson(ws.grid, M[0], I.n_i, None, E, ws)
        torch.cuda.synchronize()
        assert torch.equal(M, I.M), q
        assert torch.equal(E, E0[q]) and torch.equal(E, I.E[1]), q


def test_batch_step_matches_oracle():
    problems = SI.batched_instances(6, sizes=(8, 12), sizes_1d=(24, 32))
    b, pr = _solver(problems)
    b.step()
    for q, p in enumerate(problems):
        o = ST.Oracle(p, probes=pr[q])
        F0 = SI.initial_ht(p)
        o.efield(F0)
        Fo = o.slar_vp(F0, p.dt)
        err = normwise(b.dense(q), HT.full(Fo))
        assert err < 10 * p.tol, (q, p.n, err)


def test_tuned_configuration_keeps_the_answer():
    problems = SI.batched_instances(8, sizes=(8, 12, 16), sizes_1d=(32, 48, 64))
    b0, _ = _solver(problems)
    b0.step()
    ref = [b0.dense(q) for q in range(b0.count)]
    b1, _ = _solver(problems)
    cfg = b1.tune(reps=1)
    assert cfg["grid"] in (256, 512, 1024, 2048, 4096) and cfg["group"] in (1, 2, 4)
    assert cfg["chunk"] in (4, 8, 16)
    b1.step()
    for q, p in enumerate(problems):
        assert normwise(b1.dense(q), ref[q]) < 10 * p.tol, q


def test_batch_rejects_bad_arguments():
    p = SI.batched_instances(2)
    b, _ = _solver(p)
    bad = [L.make_adv(2, 0.1, 1.0, b.inst[q].E[0], order=5) for q in range(2)]
    with pytest.raises(L.SlarError) as e:
        b.batch.cross_update(b.state, bad, b.tol, b.rmax, b.probes,
                             [I.U for I in b.inst], [I.V for I in b.inst])
    assert e.value.status == L.SLAR_E_INVAL
    with pytest.raises(L.SlarError):
        b.batch.set_config(256, 1, 8, (4, 5, 16))


@pytest.mark.parametrize("refine", [False, True])
def test_grouped_truncation_equals_single_instance(refine):
    """The batched truncation runs each of its steps (products, Grams, sign
    rules, copies, and the single-block factorisations: Cholesky, core SVD,
    Gram eigenpairs, basis completion) as one grouped launch over all
    instances, then the frame builds; each instance must still get, bit for
    bit, the HT tensor, ranks and frames of the one-instance slar_truncate
    and slar_frames_from_ht on a workspace with the same leaf-refinement
    setting.  Factor sets of 40 to
    96 terms (the k <= 64 and k > 64 SVD forms in the same group), 1D1V and
    2D2V instances mixed; converged crosses of up to min(2 rmax, 128) terms
    reach the truncation (the rank cap applies after it)."""
    from paper_2606_29027_amd.batch import _Inst
    from gpu_util import dev, ht_from_dev
    problems = SI.batched_instances(6, sizes=(12, 16), sizes_1d=(96, 128))
    assert {p.dx for p in problems} == {1, 2}
    b, _ = _solver(problems)
    for ws in b.batch.ws:
        L.slar_leaf_refine(ws, refine)
    tol = 1e-6
    ks = [40, 80, 64, 96, 72, 50]
    keep, lrs = [], []
    for q, I in enumerate(b.inst):
        k = ks[q]
        rng = np.random.default_rng(40 + q)
        U = dev(rng.standard_normal((k, I.Nx)) * (0.8 ** np.arange(k))[:, None])
        V = dev(rng.standard_normal((k, I.Nv)))
        keep.append((U, V))
        lrs.append(L.LowRank(k, U.data_ptr(), V.data_ptr()))
    hts = [I.ht_desc(0) for I in b.inst]
    frs = [I.frames(0) for I in b.inst]
    b.batch.truncate(lrs, tol, b.rmax, hts, frs)
    torch.cuda.synchronize()
    for q, p in enumerate(problems):
        one = _Inst(p)
        H = one.ht_desc(0)
        ws = L.Workspace(L.make_grid(p), b.rmax)
        L.slar_leaf_refine(ws, refine)
        L.slar_truncate(ws.grid, lrs[q], tol, b.rmax, H, ws)
        X, P = one.frames_buf[0]
        F1 = L.slar_frames_from_ht(ws.grid, H, one.frames(0), ws)
        torch.cuda.synchronize()
        assert list(H.rank) == list(hts[q].rank), q
        # the frames built in the same grouped call
        r = F1.r
        assert frs[q].r == r, q
        Xb, Pb = b.inst[q].frames_buf[0]
        assert torch.equal(Xb[:, :r], X[:, :r]) and torch.equal(Pb[:, :r], P[:, :r]), q
        a = ht_from_dev(hts[q], b.inst[q].ht[0], p.dx + p.dv, p.n)
        c = ht_from_dev(H, one.ht[0], p.dx + p.dv, p.n)
        for key in ("root", "B12", "B34"):
            if key in a:
                assert np.array_equal(a[key], c[key]), (q, key)
        for m in range(p.dx + p.dv):
            assert np.array_equal(a["leaves"][m], c["leaves"][m]), (q, m)
