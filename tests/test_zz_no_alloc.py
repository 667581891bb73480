"""The allocation-free truncation entry point (spamm_truncate_noalloc)
against the workspace one (spamm_truncate), through the C ABI: two calls in
a row on one GPU, the second on a smaller matrix, must remove exactly the
same units and report the same removed norm; a capacity beyond the fixed
scratch array's limit is rejected before anything is enqueued."""
import ctypes
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2005_10680_amd as P  # noqa: E402


def _product(n, b, seed):
    F = oracle.BSM.of(synth.sys3d(n, seed, b))
    lmin, lmax = oracle.gerschgorin(F)
    X = oracle.x0(F, lmin, lmax)
    C, _ = oracle.spamm(X, X, 0.0, sym=True)
    return C


def _state(M):
    torch.cuda.synchronize()
    return M.brow.cpu().numpy().copy(), M.map.cpu().numpy().copy(), int(M.nslot.item())


@pytest.mark.parametrize("rel", [1e-10, 1e-6, 1e-3])
def test_noalloc_equals_workspace_truncation(rel):
    # the larger matrix first, then the smaller one: the second call reuses
    # the scratch array the first one left behind
    cases = [(2000, 64, 2), (1024, 32, 1)]
    for n, b, seed in cases:
        print(f"noalloc truncation: n={n} b={b} seed={seed} rel={rel}", flush=True)
        C = _product(n, b, seed)
        sq, _ = oracle.norms(C)
        delta = math.sqrt(float(np.sum(sq))) * rel
        M1 = P.BlockSparse.from_host(C)
        M2 = P.BlockSparse.from_host(C)
        P.build_norms(M1)
        P.build_norms(M2)
        out1 = P.truncate(M1, delta)
        out2 = P.truncate_noalloc(M2, delta)
        torch.cuda.synchronize()
        b1, m1, s1 = _state(M1)
        b2, m2, s2 = _state(M2)
        assert s1 == s2
        assert np.array_equal(b1, b2)
        assert np.array_equal(m1, m2)
        o1 = out1.cpu().numpy()
        o2 = out2.cpu().numpy()
        assert np.array_equal(o1.view(np.uint64), o2.view(np.uint64))
        # and both equal the oracle's removed set
        Ot, info = oracle.truncate(C, delta)
        brow, bcol, vals, _, _, _ = M2.live()
        assert np.array_equal(oracle.BSM(M2.n, M2.b, brow, bcol, vals).keys(), Ot.keys())
        assert int(o2[0]) == info.removed_keys.shape[0]


def test_noalloc_rejects_capacity_beyond_limit():
    lim = int(P.lib().spamm_truncate_noalloc_max_cap())
    assert lim == 1 << 20
    C = _product(1024, 32, 1)
    M = P.BlockSparse.from_host(C)
    P.build_norms(M)
    torch.cuda.synchronize()
    before = M.brow.cpu().numpy().copy()
    st = M.struct()
    fake = P.spamm_bsm(st.n, st.b, st.nb, lim + 1, st.nslot, st.brow, st.bcol, st.map, st.val, st.norm, st.sq,
                       st.sqlo)
    rc = P.lib().spamm_truncate_noalloc(ctypes.byref(fake), 1e-3, P.SYNC, None, None)
    assert rc == P.SPAMM_EINVAL
    assert b"limit" in P.lib().spamm_last_error()
    # nothing was enqueued
    torch.cuda.synchronize()
    assert np.array_equal(before, M.brow.cpu().numpy())
