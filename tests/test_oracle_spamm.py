"""Pins of the oracle's SpAMM product (Algorithm 2 at the leaf level),
truncation, traces and starting matrix.

* kept set == brute-force enumeration of every (i, k, j);
* tau = 0 reproduces the dense product A @ B;
* tau > 0 equals the dense sum over the kept triples;
* symmetric mode (i <= j, mirrored) equals the full computation bit for bit;
* truncation: ||E||_F < delta recomputed exactly, maximality, symmetry;
* traces and Gerschgorin bounds against numpy / eigvalsh."""
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import synth


def rand_bsm(rng, nb, b, density, decay=0.5, zero_blocks=0.0, n=None, sym=False):
    if n is None:
        n = nb * b - int(rng.integers(0, b))
    D = np.zeros((nb * b, nb * b))
    present = rng.random((nb, nb)) < density
    present[np.arange(nb), np.arange(nb)] = True
    if sym:
        present = present | present.T
    for r, c in zip(*np.nonzero(present)):
        blk = rng.standard_normal((b, b)) * math.exp(-decay * abs(r - c)) * math.exp(rng.uniform(-8, 0))
        if rng.random() < zero_blocks:
            blk[:] = 0.0
        D[r*b:(r+1)*b, c*b:(c+1)*b] = blk
    D = D[:n, :n]
    if sym:
        D = (D + D.T) / 2
    M = oracle.from_dense(D, b)
    return M


def brute_kept(A, B, tau, sym):
    nb = A.nb
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    mA, mB = A.block_map(), B.block_map()
    out = set()
    for i in range(nb):
        for j in range(nb):
            if sym and i > j:
                continue
            for k in range(nb):
                sa, sb = mA[i*nb+k], mB[k*nb+j]
                if sa >= 0 and sb >= 0 and nuA[sa] * nuB[sb] >= tau:
                    out.add((i, k, j))
    return out


def kept_set(K):
    s = set()
    for m in range(K.oi.shape[0]):
        for q in range(K.kptr[m], K.kptr[m+1]):
            s.add((int(K.oi[m]), int(K.klist[q]), int(K.oj[m])))
    return s


def padded(M):
    nb, b = M.nb, M.b
    P = np.zeros((nb * b, nb * b))
    P[:M.n, :M.n] = M.to_dense()
    return P


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("sym", [False, True])
def test_kept_set_bruteforce(seed, sym):
    rng = np.random.default_rng(seed)
    nb = [3, 4, 5, 6, 7][seed]
    A = rand_bsm(rng, nb, 3, 0.5, zero_blocks=0.1, sym=sym)
    B = A if sym else rand_bsm(rng, nb, 3, 0.5, zero_blocks=0.1, n=A.n)
    _, nuA = oracle.norms(A)
    ps = sorted(set(nuA))
    for tau in [0.0, ps[len(ps)//3] ** 2, ps[-1] ** 2 * 0.5, 1e300]:
        K = oracle.kept(A, B, tau, sym)
        assert kept_set(K) == brute_kept(A, B, tau, sym)
        assert np.all(np.diff(K.klist[K.kptr[0]:K.kptr[1]]) > 0) if K.oi.shape[0] else True


@pytest.mark.parametrize("seed", range(4))
def test_tau_zero_is_dense_product(seed):
    rng = np.random.default_rng(20 + seed)
    A = rand_bsm(rng, 5, 4, 0.6)
    B = rand_bsm(rng, 5, 4, 0.6, n=A.n)
    C, K = oracle.spamm(A, B, 0.0)
    ref = A.to_dense() @ B.to_dense()
    got = C.to_dense()
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    # every present triple is kept
    nb = A.nb
    assert K.npairs == sum(1 for (i, k, j) in brute_kept(A, B, 0.0, False))


@pytest.mark.parametrize("seed", range(4))
def test_spamm_equals_sum_of_kept_products(seed):
    rng = np.random.default_rng(40 + seed)
    A = rand_bsm(rng, 6, 3, 0.7)
    B = rand_bsm(rng, 6, 3, 0.7, n=A.n)
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    tau = float(np.median(nuA)) * float(np.median(nuB))
    C, K = oracle.spamm(A, B, tau)
    Ap, Bp = padded(A), padded(B)
    b = A.b
    ref = np.zeros_like(Ap)
    for (i, k, j) in brute_kept(A, B, tau, False):
        ref[i*b:(i+1)*b, j*b:(j+1)*b] += Ap[i*b:(i+1)*b, k*b:(k+1)*b] @ Bp[k*b:(k+1)*b, j*b:(j+1)*b]
    np.testing.assert_allclose(padded(C), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    # the guarantee of the selection: error below the bound of Algorithm 3
    err = np.linalg.norm(Ap @ Bp - padded(C))
    bound = oracle.cse_tree(A, B, np.array([tau]))[0]
    assert err <= bound * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_symmetric_mode_bitwise(seed):
    rng = np.random.default_rng(60 + seed)
    X = rand_bsm(rng, 6, 4, 0.5, sym=True)
    _, nu = oracle.norms(X)
    tau = float(np.quantile(nu, 0.3)) ** 2
    Cs, Ks = oracle.spamm(X, X, tau, sym=True)
    Cf, Kf = oracle.spamm(X, X, tau, sym=False)
    assert np.array_equal(Cs.keys(), Cf.keys())
    assert np.array_equal(Cs.vals, Cf.vals)           # same products, same order
    D = Cs.to_dense()
    assert np.array_equal(D, D.T)


@settings(max_examples=40, deadline=None)
@given(nb=st.integers(1, 6), b=st.sampled_from([1, 2, 3, 4]), seed=st.integers(0, 10**6),
       dens=st.floats(0.1, 1.0), qt=st.floats(0.0, 1.0))
def test_property_bound_and_kept(nb, b, seed, dens, qt):
    rng = np.random.default_rng(seed)
    A = rand_bsm(rng, nb, b, dens, zero_blocks=0.15)
    B = rand_bsm(rng, nb, b, dens, zero_blocks=0.15, n=A.n)
    if A.n == 0:
        return
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    ps = np.outer(nuA, nuB).ravel()
    tau = float(np.quantile(ps, qt)) if ps.size else 0.0
    C, K = oracle.spamm(A, B, tau)
    assert kept_set(K) == brute_kept(A, B, tau, False)
    err = np.linalg.norm(padded(A) @ padded(B) - padded(C))
    bound = oracle.cse_tree(A, B, np.array([tau if tau > 0 else 1e-300]))[0]
    flat, ssum = oracle.cse_flat_sum(A, B, np.array([tau if tau > 0 else 1e-300]))
    # slack for the rounding of two different dense evaluations of the product
    slack = 1e-13 * np.linalg.norm(padded(A)) * np.linalg.norm(padded(B))
    assert err <= flat[0] * (1 + 1e-12) + slack
    assert flat[0] <= bound * (1 + 1e-12) + 1e-300
    assert bound <= ssum[0] * (1 + 1e-12) + 1e-300


# ---------------------------------------------------------------------------
# truncation
# ---------------------------------------------------------------------------

def exact_fro2(vals) -> Fraction:
    return sum((Fraction(float(x)) ** 2 for x in np.ravel(vals)), Fraction(0))


@pytest.mark.parametrize("seed", range(5))
def test_truncation_error_below_delta_and_maximal(seed):
    rng = np.random.default_rng(80 + seed)
    X = rand_bsm(rng, 8, 3, 0.6, decay=0.9, sym=True, zero_blocks=0.05)
    sq, nu = oracle.norms(X)
    total = float(np.sqrt(np.sum(sq)))
    for delta in [total * 1e-9, total * 1e-3, total * 0.05, total * 0.3]:
        Xt, info = oracle.truncate(X, delta)
        removed = ~np.isin(X.keys(), Xt.keys())
        E2 = exact_fro2(X.vals[removed])
        assert E2 < Fraction(delta) ** 2                      # ||E||_F < delta, exactly
        D = Xt.to_dense()
        assert np.array_equal(D, D.T)                          # symmetric units
        # maximality: the next unit in the rule's order would break the budget
        up = X.brow <= X.bcol
        w = np.where(X.brow[up] == X.bcol[up], 1.0, 2.0)
        T, Q, kt = oracle.trunc_quanta(delta)
        k = oracle.trunc_keys(sq[up], w, Q)
        order = np.lexsort((X.keys()[up], k))
        q = info.removed_keys.shape[0]
        assert set(X.keys()[up][order[:q]]) == set(info.removed_keys)
        if q < order.shape[0]:
            assert int(np.sum(k[order[:q+1]].astype(object))) >= kt
        # quantised keys never undercount: k*Q >= w*sq
        ns = k < oracle.KSAT                                   # saturated keys are never removable
        assert np.all(k[ns].astype(np.float64) * Q >= (w * sq[up])[ns])
        assert np.all((w * sq[up])[~ns] >= oracle.KSAT * Q)


def test_truncation_zero_blocks_and_extremes():
    rng = np.random.default_rng(3)
    X = rand_bsm(rng, 5, 2, 0.8, sym=True)
    Xz = oracle.BSM(X.n, X.b, X.brow, X.bcol, X.vals.copy())
    zero_blk = np.nonzero(Xz.brow == Xz.bcol)[0][0]
    Xz.vals[zero_blk] = 0.0
    Xt, info = oracle.truncate(Xz, 1e-100)
    assert Xz.keys()[zero_blk] not in set(Xt.keys())          # a zero block is free to drop
    Xt, info = oracle.truncate(X, 0.0)
    assert Xt.nblk == X.nblk                                   # delta = 0 removes nothing
    big = 2.0 * np.linalg.norm(X.to_dense())
    Xt, info = oracle.truncate(X, big)
    assert Xt.nblk == 0                                        # everything fits the budget


# ---------------------------------------------------------------------------
# traces, Gerschgorin, starting matrix
# ---------------------------------------------------------------------------

def test_traces_exact():
    rng = np.random.default_rng(4)
    X = rand_bsm(rng, 5, 4, 0.7, sym=True)
    t1, t2, e = oracle.traces(X)
    D = X.to_dense()
    assert t1 == math.fsum(np.diag(D))
    F2 = exact_fro2(D)
    assert t2 == F2.numerator / F2.denominator
    ex = sum((Fraction(float(x)) for x in np.diag(D)), Fraction(0)) - F2
    assert e == ex.numerator / ex.denominator


def test_gerschgorin_and_x0():
    F = oracle.BSM.of(synth.chain1d(256, 1, 32))
    lmin, lmax = oracle.gerschgorin(F)
    D = F.to_dense()
    w = np.linalg.eigvalsh(D)
    assert lmin <= w[0] and w[-1] <= lmax
    R = np.sum(np.abs(D), axis=1) - np.abs(np.diag(D))
    assert lmin == pytest.approx(np.min(np.diag(D) - R), rel=1e-15)
    assert lmax == pytest.approx(np.max(np.diag(D) + R), rel=1e-15)
    X0 = oracle.x0(F, lmin, lmax)
    ref = (lmax * np.eye(F.n) - D) / (lmax - lmin)
    np.testing.assert_allclose(X0.to_dense(), ref, rtol=1e-15, atol=1e-17)
    wx = np.linalg.eigvalsh(X0.to_dense())
    assert wx[0] >= -1e-14 and wx[-1] <= 1 + 1e-14
    # every diagonal block present
    assert all(X0.block_map()[d * X0.nb + d] >= 0 for d in range(X0.nb))
