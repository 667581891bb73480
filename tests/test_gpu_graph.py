"""The graph-captured purification loop (decisions on the device, the step
replayed as one HIP graph) against the oracle and against the host-driven
loop: an FP64 graph run takes the oracle's decisions at every step and
ends within 1e-12 of its result (each of Algorithms 5, 4 and 1); with the
FP32 and split-BF16 tiers each step is checked against the oracle from the
GPU's own iterate (the host loop makes the split-BF16 copies on a side
stream beside the sweeps, the graph on its one stream).  Same kernels and decisions as the host loop, so results and every
per-iteration record are identical bit for bit.  The graph is replayed many
times within one run and the run is repeated with eager host-loop work in
between."""
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


def system(case):
    if case == "chain":
        Fm = synth.chain1d(1024, 1, 32)
        n_occ, taus = 512, synth.tau_paper()
    else:
        Fm = synth.sys3d(2000, 5, 64)
        n_occ, taus = 1000, synth.tau_log(32)
    w = np.linalg.eigvalsh(oracle.BSM.of(Fm).to_dense())
    return Fm, n_occ, taus, w[n_occ - 1], w[n_occ]


def same(r1, r2):
    assert len(r1.logs) == len(r2.logs)
    for a, b in zip(r1.logs, r2.logs):
        for f in FIELDS:
            assert a[f] == b[f], (f, a["i"], a[f], b[f])
    b1, c1, v1, _, _, _ = r1.D.live()
    b2, c2, v2, _, _, _ = r2.D.live()
    assert np.array_equal(b1, b2) and np.array_equal(c1, c2)
    assert np.array_equal(v1, v2)


@pytest.mark.parametrize("case,variant,precision", [
    ("chain", "hybrid", "fp64"), ("chain", "spamm", "fp64"), ("chain", "truncmul", "fp64"),
    ("sys3d", "hybrid", "fp64"), ("sys3d", "hybrid", "fp32"), ("sys3d", "hybrid", "bf16x3")])
def test_graph_loop_matches_host_loop(case, variant, precision):
    Fm, n_occ, taus, homo, lumo = system(case)
    F = P.BlockSparse.from_host(Fm)
    kw = dict(homo=homo, lumo=lumo, variant=variant, precision=precision)
    host = P.purify(F, n_occ, 1e-6, taus, **kw)
    g1 = P.purify(F, n_occ, 1e-6, taus, graph_steps=4, **kw)
    same(host, g1)
    assert host.status == g1.status
    # eager host-loop work between two graph runs, then other poll intervals
    host2 = P.purify(F, n_occ, 1e-6, taus, **kw)
    same(host, host2)
    for k in (1, 100):
        gk = P.purify(F, n_occ, 1e-6, taus, graph_steps=k, **kw)
        same(host, gk)
    assert sum(1 for lg in host.logs if lg["branch"] >= 0) >= 8
    # against the oracle
    p = oc.params(n_occ, taus, homo, lumo, variant=variant, precision=precision)
    if precision == "fp64":
        oc.end_to_end(Fm, p, g1.logs, g1.D)
    else:
        taped = P.purify(F, n_occ, 1e-6, taus, keep_tape=True, **kw)
        same(taped, g1)
        assert oc.teacher_forced(Fm, p, taped) > 0


def test_graph_loop_n_max_warning():
    Fm, n_occ, taus, homo, lumo = system("chain")
    F = P.BlockSparse.from_host(Fm)
    host = P.purify(F, n_occ, 1e-6, taus, homo=homo, lumo=lumo, n_max=5)
    g = P.purify(F, n_occ, 1e-6, taus, homo=homo, lumo=lumo, n_max=5, graph_steps=3)
    assert host.status == P.SPAMM_WNOCONV == g.status
    same(host, g)


def test_capacity_error_in_both_loops():
    Fm, n_occ, taus, homo, lumo = system("chain")
    F = P.BlockSparse.from_host(Fm)
    for gs in (0, 2):
        with pytest.raises(P.SpammError) as ei:
            P.purify(F, n_occ, 1e-6, taus, homo=homo, lumo=lumo, max_pairs=64, graph_steps=gs)
        assert ei.value.code == P.SPAMM_ECAPACITY
    # the library still works afterwards
    r = P.purify(F, n_occ, 1e-6, taus, homo=homo, lumo=lumo, graph_steps=2)
    assert r.status == P.SPAMM_OK


def test_graph_mode_rejects_tape():
    Fm, n_occ, taus, homo, lumo = system("chain")
    F = P.BlockSparse.from_host(Fm)
    with pytest.raises(P.SpammError) as ei:
        P.purify(F, n_occ, 1e-6, taus, homo=homo, lumo=lumo, keep_tape=True, graph_steps=2)
    assert ei.value.code == P.SPAMM_EINVAL
