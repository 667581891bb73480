"""Batched purification (independent systems, one persistent product launch
per leaf size and tier per step): every system's result and per-iteration
records are bit-identical to its own single-system run, and every system is
checked against the oracle -- FP64 systems end to end (the oracle's
decisions at every step, result within 1e-12), tier systems step by step
from the GPU's own iterates; systems stop at different iterations; a
failing system leaves the others intact."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import oracle_checks as oc  # noqa: E402
import paper_2005_10680_amd as P  # noqa: E402

FIELDS = ["i", "branch", "idx", "stop", "delta", "tau", "t1", "t2", "e", "npairs", "nout", "nslot_hat",
          "nslot_kept", "removed_units", "removed_fro2", "npairs_low", "sigma", "sidx"]


def make(kind, n, b, seed):
    Fm = synth.chain1d(n, seed, b) if kind == "chain" else synth.sys3d(n, seed, b)
    w, U = np.linalg.eigh(oracle.BSM.of(Fm).to_dense())
    taus = synth.tau_paper() if kind == "chain" else synth.tau_log(32)
    return Fm, n // 2, taus, w[n // 2 - 1], w[n // 2], U


def same_logs(la, lb):
    assert len(la) == len(lb)
    for a, b in zip(la, lb):
        for f in FIELDS:
            assert a[f] == b[f], (f, a["i"], a[f], b[f])


def same_matrix(A, B):
    b1, c1, v1, n1, s1, _ = A.live()
    b2, c2, v2, n2, s2, _ = B.live()
    assert np.array_equal(b1, b2) and np.array_equal(c1, c2)
    assert np.array_equal(v1, v2)
    assert np.array_equal(n1.view(np.uint64), n2.view(np.uint64))
    assert np.array_equal(s1.view(np.uint64), s2.view(np.uint64))


def exact_norms(M):
    """The block norms M holds (taken in the product epilogue) are the
    exactly rounded norms of its values."""
    brow, bcol, vals, nrm, sq, _ = M.live()
    osq, onu = oracle.norms(oracle.BSM(M.n, M.b, brow, bcol, vals))
    assert np.array_equal(sq.view(np.uint64), osq.view(np.uint64))
    assert np.array_equal(nrm.view(np.uint64), onu.view(np.uint64))


SYSTEMS = [("sys3d", 1000, 64, 11, "hybrid", "fp64"), ("sys3d", 2048, 64, 12, "hybrid", "fp64"),
           ("chain", 1024, 32, 1, "hybrid", "fp64"), ("sys3d", 1536, 32, 13, "spamm", "fp64"),
           ("sys3d", 2500, 64, 14, "hybrid", "fp32"), ("chain", 768, 32, 2, "truncmul", "fp64")]


def test_batch_matches_single_runs():
    data = [make(k, n, b, sd) for k, n, b, sd, _, _ in SYSTEMS]
    Fs = [P.BlockSparse.from_host(d[0]) for d in data]
    variants = [s[4] for s in SYSTEMS]
    precs = [s[5] for s in SYSTEMS]
    res = P.purify_batched(Fs, [d[1] for d in data], 1e-6, [d[2] for d in data], [d[3] for d in data],
                           [d[4] for d in data], variant=variants, precision=precs, graph_steps=4)
    assert res.rc == P.SPAMM_OK and all(st == P.SPAMM_OK for st in res.status)
    iters = []
    for q, (d, F) in enumerate(zip(data, Fs)):
        single = P.purify(F, d[1], 1e-6, d[2], homo=d[3], lumo=d[4], variant=variants[q], precision=precs[q],
                          keep_tape=precs[q] != "fp64")
        same_logs(single.logs, res.logs[q])
        same_matrix(single.D, res.D[q])
        exact_norms(res.D[q])
        iters.append(len(res.logs[q]))
        oracle_check(d, variants[q], precs[q], res.logs[q], res.D[q], single)
    assert len(set(iters)) > 1          # the systems stop at different iterations
    # converged against the dense eigensolver
    for q in (0, 2):
        d = data[q]
        U = d[5]
        Dref = U[:, :d[1]] @ U[:, :d[1]].T
        brow, bcol, vals, _, _, _ = res.D[q].live()
        Dg = oracle.BSM(Fs[q].n, Fs[q].b, brow, bcol, vals).to_dense()
        assert np.linalg.norm(Dg - Dref) < 1e-6


def oracle_check(d, variant, prec, logs, D, single):
    """System d of a batch against the oracle: FP64 end to end; a tier
    system step by step on its single run's tape (bit-identical to the
    batched run)."""
    p = oc.params(d[1], d[2], d[3], d[4], variant=variant, precision=prec)
    if prec == "fp64":
        oc.end_to_end(d[0], p, logs, D)
    else:
        oc.teacher_forced(d[0], p, single)


def test_batch_isolates_a_failing_system():
    data = [make("sys3d", 1000, 64, 21), make("chain", 1024, 32, 3), make("sys3d", 1200, 64, 22)]
    Fs = [P.BlockSparse.from_host(d[0]) for d in data]
    mp = [None, 64, None]
    mp = [m if m is not None else F.nb * F.nb * (F.nb + 1) // 2 for m, F in zip(mp, Fs)]
    res = P.purify_batched(Fs, [d[1] for d in data], 1e-6, [d[2] for d in data], [d[3] for d in data],
                           [d[4] for d in data], max_pairs=mp, graph_steps=2, raise_on_error=False)
    assert res.status[1] == P.SPAMM_ECAPACITY and res.rc == P.SPAMM_ECAPACITY
    for q in (0, 2):
        assert res.status[q] == P.SPAMM_OK
        d = data[q]
        single = P.purify(Fs[q], d[1], 1e-6, d[2], homo=d[3], lumo=d[4])
        same_logs(single.logs, res.logs[q])
        same_matrix(single.D, res.D[q])


def test_batch_all_product_groups():
    """Seven systems, one in each product group (leaf 32, 64, 128 in FP64;
    leaf 32 and 64 in the FP32 and split-BF16 tiers): every system equals
    its own single run."""
    specs = [(32, "fp64"), (64, "fp64"), (128, "fp64"), (32, "fp32"), (64, "fp32"), (32, "bf16x3"), (64, "bf16x3")]
    data, Fs, precs = [], [], []
    for t, (b, prec) in enumerate(specs):
        d = make("sys3d", 900 + 37 * t, b, 40 + t)
        data.append(d)
        Fs.append(P.BlockSparse.from_host(d[0]))
        precs.append(prec)
    res = P.purify_batched(Fs, [d[1] for d in data], 1e-6, [d[2] for d in data], [d[3] for d in data],
                           [d[4] for d in data], precision=precs, graph_steps=4)
    assert res.rc == P.SPAMM_OK
    for q, (d, F) in enumerate(zip(data, Fs)):
        single = P.purify(F, d[1], 1e-6, d[2], homo=d[3], lumo=d[4], precision=precs[q],
                          keep_tape=precs[q] != "fp64")
        same_logs(single.logs, res.logs[q])
        same_matrix(single.D, res.D[q])
        oracle_check(d, "hybrid", precs[q], res.logs[q], res.D[q], single)
