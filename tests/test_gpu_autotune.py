"""Re-blocking, the product schedule and the leaf-size autotuner.

* re-blocking keeps the matrix: the dense matrix of the result equals the
  input's bit for bit (ragged n, up and down the leaf sizes), the block
  pattern is the structural one, and the norms equal the oracle's;
* the schedule (workgroups per CU) never changes results;
* the autotuner picks a leaf size it tried and the purification at that
  leaf size converges."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2005_10680_amd as P  # noqa: E402


def to_oracle(M):
    brow, bcol, vals, _, _, _ = M.live()
    return oracle.BSM(M.n, M.b, brow, bcol, vals)


def test_reblock_roundtrip_and_norms():
    Fm = synth.sys3d(1000, 31, 32)             # ragged: 1000 = 31 * 32 + 8
    F = P.BlockSparse.from_host(Fm)
    dense = oracle.BSM.of(Fm).to_dense()
    for b in (64, 128, 32):
        Y = P.reblock(F, b)
        Yo = to_oracle(Y)
        assert np.array_equal(Yo.to_dense(), dense)
        # structural pattern: (R, C) present iff an overlapping leaf-32 block is
        nbY = Y.nb
        pres = set(zip(Yo.brow.tolist(), Yo.bcol.tolist()))
        want = set()
        for r, c in zip(Fm.brow.tolist(), Fm.bcol.tolist()):
            want.add((r * 32 // b, c * 32 // b))
        assert pres == {k for k in want if k[0] < nbY and k[1] < nbY}
        # norms of the result equal the oracle's exactly rounded norms
        _, _, _, nrm, _, _ = Y.live()
        assert np.array_equal(nrm, oracle.norms(Yo)[1])
    # and back down from 128 to 32
    Y128 = P.reblock(F, 128)
    Z = P.reblock(Y128, 32)
    assert np.array_equal(to_oracle(Z).to_dense(), dense)


def test_schedule_does_not_change_results():
    Fm = synth.sys3d(2000, 5, 64)
    F0 = oracle.BSM.of(Fm)
    w = np.linalg.eigvalsh(F0.to_dense())
    F = P.BlockSparse.from_host(Fm)
    ref = P.purify(F, 1000, 1e-6, synth.tau_log(32), homo=w[999], lumo=w[1000])
    default = P.get_gemm_schedule(64)
    try:
        for pc in (1, 2):
            P.set_gemm_schedule(64, pc)
            assert P.get_gemm_schedule(64) == pc
            r = P.purify(F, 1000, 1e-6, synth.tau_log(32), homo=w[999], lumo=w[1000])
            a, b_ = ref.D.live(), r.D.live()
            assert np.array_equal(a[0], b_[0]) and np.array_equal(a[1], b_[1]) and np.array_equal(a[2], b_[2])
    finally:
        P.set_gemm_schedule(64, 0)
    assert P.get_gemm_schedule(64) == default


def test_autotune_picks_a_working_leaf():
    n = 2048
    Fm = synth.sys3d(n, 8, 32)
    F0 = oracle.BSM.of(Fm)
    w, U = np.linalg.eigh(F0.to_dense())
    F = P.BlockSparse.from_host(Fm)
    taus = synth.tau_log(32)
    saved = {b: P.get_gemm_schedule(b) for b in (32, 64, 128)}
    try:
        b, pc, ms = P.autotune(F, n // 2, 1e-6, taus, homo=w[n // 2 - 1], lumo=w[n // 2], trial_steps=5)
        assert set(ms) == {32, 64, 128} and all(v > 0 for v in ms.values())
        assert b == min(ms, key=ms.get)
        assert 1 <= pc <= saved[b] and P.get_gemm_schedule(b) == pc
        Fb = P.reblock(F, b)
        r = P.purify(Fb, n // 2, 1e-6, taus, homo=w[n // 2 - 1], lumo=w[n // 2])
        Dref = U[:, :n // 2] @ U[:, :n // 2].T
        assert np.linalg.norm(to_oracle(r.D).to_dense() - Dref) < 1e-6
    finally:
        for bb, v in saved.items():
            P.set_gemm_schedule(bb, v)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_autotune_precision_tiers_skip_leaf_128(precision):
    """The precision tiers run at leaf 32 and 64 only: their trials leave
    leaf 128 out (no time reported for it) and the chosen leaf purifies in
    that tier."""
    n = 2048
    Fm = synth.sys3d(n, 9, 32)
    w = np.linalg.eigvalsh(oracle.BSM.of(Fm).to_dense())
    F = P.BlockSparse.from_host(Fm)
    taus = synth.tau_log(32)
    saved = {b: P.get_gemm_schedule(b) for b in (32, 64, 128)}
    try:
        b, pc, ms = P.autotune(F, n // 2, 1e-6, taus, homo=w[n // 2 - 1], lumo=w[n // 2], precision=precision,
                               trial_steps=4)
        assert set(ms) == {32, 64} and all(v > 0 for v in ms.values())
        assert b == min(ms, key=ms.get) and 1 <= pc <= saved[b]
        r = P.purify(P.reblock(F, b), n // 2, 1e-6, taus, homo=w[n // 2 - 1], lumo=w[n // 2], precision=precision)
        assert r.status >= 0 and sum(lg["npairs_low"] for lg in r.logs) > 0
    finally:
        for bb, v in saved.items():
            P.set_gemm_schedule(bb, v)
