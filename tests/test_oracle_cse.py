"""Pins of the oracle's error bound (Algorithm 3) and selection rule.

* the paper's worked 2x2 example, eqs. (3)-(6) (fixture under golden/);
* the closed form at nb = 2 for threshold-defined skip sets;
* brute force: an independent bottom-up evaluation over a dense array of
  leaf errors, and the true SpAMM error measured with dense products;
* orderings  measured <= B_flat <= B_tree <= B_sum,  monotonicity, the
  zero and all-skipped cases (the bound ||A||_F ||B||_F of the text after
  eq. (3))."""
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_bsm(rng, nb, b, density, decay=0.0, sym=False, zero_blocks=0.0, n=None):
    if n is None:
        n = nb * b - int(rng.integers(0, b))  # ragged tail
    present = rng.random((nb, nb)) < density
    present[np.arange(nb), np.arange(nb)] = True
    if sym:
        present = present | present.T
    rr, cc = np.nonzero(present)
    vals = rng.standard_normal((rr.shape[0], b, b))
    scale = np.exp(-decay * np.abs(rr - cc))
    vals *= scale[:, None, None]
    zb = rng.random(rr.shape[0]) < zero_blocks
    vals[zb] = 0.0
    M = oracle.BSM(n, b, rr.astype(np.int32), cc.astype(np.int32), vals)
    D = M.to_dense()
    if sym:
        D = (D + D.T) / 2
        M = oracle.from_dense(D, b)
        # keep structural pattern symmetric even where values vanish
    else:
        # zero padding rows/cols
        M = oracle.from_dense(D, b)
    return M


def dense_spamm_error(A, B, tau):
    """||AB - SpAMM(A,B,tau)||_F from dense per-triple products."""
    nb, b = A.nb, A.b
    Ad = np.zeros((nb * b, nb * b)); Ad[:A.n, :A.n] = A.to_dense()
    Bd = np.zeros((nb * b, nb * b)); Bd[:B.n, :B.n] = B.to_dense()
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    mA, mB = A.block_map(), B.block_map()
    E = np.zeros_like(Ad)
    for i in range(nb):
        for j in range(nb):
            for k in range(nb):
                sa, sb = mA[i * nb + k], mB[k * nb + j]
                if sa < 0 or sb < 0:
                    continue
                if nuA[sa] * nuB[sb] < tau:
                    E[i*b:(i+1)*b, j*b:(j+1)*b] += Ad[i*b:(i+1)*b, k*b:(k+1)*b] @ Bd[k*b:(k+1)*b, j*b:(j+1)*b]
    return np.linalg.norm(E)


def bottom_up_bound(A, B, tau):
    """Independent evaluation of Algorithm 3: a dense (P,P,P) array of leaf
    errors reduced level by level with numpy slicing."""
    nb = A.nb
    P = 1
    while P < nb:
        P *= 2
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    mA, mB = A.block_map(), B.block_map()
    e = np.zeros((P, P, P))
    for i in range(nb):
        for k in range(nb):
            sa = mA[i * nb + k]
            if sa < 0:
                continue
            for j in range(nb):
                sb = mB[k * nb + j]
                if sb < 0:
                    continue
                p = nuA[sa] * nuB[sb]
                if p < tau:
                    e[i, k, j] = p
    while e.shape[0] > 1:
        h = e.shape[0] // 2
        acc = np.zeros((h, h, h))
        for a in (0, 1):
            for c in (0, 1):
                t = e[a::2, 0::2, c::2] + e[a::2, 1::2, c::2]
                acc = acc + t * t
        e = np.sqrt(acc)
    return float(e[0, 0, 0])


# ---------------------------------------------------------------------------
# worked example, eqs. (3)-(6)
# ---------------------------------------------------------------------------

def _paper_label(lbl):
    """'A10' -> ('A', row 0, col 1): X_pq sits at block row q, column p (eq. (2))."""
    return lbl[0], int(lbl[2]), int(lbl[1])


def test_worked_example_eqs_3_to_6():
    fx = json.load(open(os.path.join(GOLD, "worked_example_eq3_6.json")))
    rng = np.random.default_rng(5)
    b = 3
    A = oracle.BSM(2 * b, b, np.array([0, 0, 1, 1], np.int32), np.array([0, 1, 0, 1], np.int32),
                   rng.standard_normal((4, b, b)) * np.array([1.0, 0.3, 2.0, 0.5])[:, None, None])
    B = oracle.BSM(2 * b, b, np.array([0, 0, 1, 1], np.int32), np.array([0, 1, 0, 1], np.int32),
                   rng.standard_normal((4, b, b)) * np.array([0.7, 1.5, 0.2, 1.1])[:, None, None])
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    mA, mB = A.block_map(), B.block_map()

    def blk(M, r, c):
        return M.vals[M.block_map()[r * 2 + c]].T

    def prod(lbl):  # 'A10B01' -> dense block product
        _, ra, ca = _paper_label(lbl[:3])
        _, rb, cb = _paper_label(lbl[3:])
        assert ca == rb
        return blk(A, ra, ca) @ blk(B, rb, cb), (ra, ca, cb)

    # leaf errors: p for the skipped products of the fixture, 0 otherwise
    lv = np.zeros((2, 2, 2))
    for lbl in fx["skipped"]:
        _, (i, k, j) = prod(lbl)
        lv[i, k, j] = nuA[mA[i * 2 + k]] * nuB[mB[k * 2 + j]]
    got = oracle.cse_tree_leafvals(A, B, lv)

    # eq. (6) evaluated exactly, from the fixture's grouping
    getcontext().prec = 60
    tot = Fraction(0)
    for grp in fx["bound_groups"]:
        s = Fraction(0)
        for lbl in grp:
            _, (i, k, j) = prod(lbl)
            s += Fraction(float(nuA[mA[i * 2 + k]])) * Fraction(float(nuB[mB[k * 2 + j]]))
        tot += s * s
    exact = float(Decimal(tot.numerator) / Decimal(tot.denominator)) ** 0.5
    exact = float((Decimal(tot.numerator) / Decimal(tot.denominator)).sqrt())
    assert abs(got - exact) <= 4 * math.ulp(exact)

    # eq. (4): the approximate product keeps exactly the listed terms, and
    # eq. (5): the error matrix holds the skipped ones
    kept_triples = set()
    for key, terms in fx["C_tilde"].items():
        for lbl in terms:
            kept_triples.add(prod(lbl)[1])
    K = oracle.Kept(np.array([0, 0, 1, 1], np.int32), np.array([0, 1, 0, 1], np.int32),
                    np.zeros(5, np.int64), np.zeros(0, np.int32))
    kl, kp = [], [0]
    for (oi, oj) in [(0, 0), (0, 1), (1, 0), (1, 1)]:
        ks = sorted(k for (i, k, j) in kept_triples if (i, j) == (oi, oj))
        kl += ks; kp.append(len(kl))
    K.kptr = np.array(kp, np.int64); K.klist = np.array(kl, np.int32)
    Ct = oracle.block_products(A, B, K)
    Ad, Bd = A.to_dense(), B.to_dense()
    C = Ad @ Bd
    Cts = np.zeros_like(C)
    for m, (oi, oj) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        Cts[oi*b:(oi+1)*b, oj*b:(oj+1)*b] = Ct[m].T
    for key, terms in fx["C_tilde"].items():
        # fixture keys are paper labels 'pq': block row q, column p
        r, c = int(key[1]), int(key[0])
        want = sum((prod(l)[0] for l in terms), np.zeros((b, b)))
        np.testing.assert_allclose(Cts[r*b:(r+1)*b, c*b:(c+1)*b], want, rtol=1e-14, atol=1e-14)
    E = C - Cts
    for key, terms in fx["E"].items():
        r, c = int(key[1]), int(key[0])
        want = sum((prod(l)[0] for l in terms), np.zeros((b, b)))
        np.testing.assert_allclose(E[r*b:(r+1)*b, c*b:(c+1)*b], want, rtol=1e-13, atol=1e-13)
    assert np.linalg.norm(E) <= got


def test_worked_example_skip_set_is_not_a_threshold_set():
    """The example's skip set would need nu(B01) < nu(B11) and nu(B11) < nu(B01)
    at once, so no single threshold produces it; the bound's combination
    rule is pinned through explicit leaf errors above."""
    fx = json.load(open(os.path.join(GOLD, "worked_example_eq3_6.json")))
    skipped = {(l[:3], l[3:]) for l in fx["skipped"]}
    # A10 B01 skipped while A10 B11 kept -> nu(B01) < nu(B11)
    assert ("A10", "B01") in skipped and ("A10", "B11") not in skipped
    # A11 B11 skipped while A11 B01 kept -> nu(B11) < nu(B01)
    assert ("A11", "B11") in skipped and ("A11", "B01") not in skipped


# ---------------------------------------------------------------------------
# closed form at nb = 2 and brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_nb2_closed_form(seed):
    rng = np.random.default_rng(100 + seed)
    A = rand_bsm(rng, 2, 4, 1.0)
    B = rand_bsm(rng, 2, 4, 1.0, n=A.n)
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    mA, mB = A.block_map(), B.block_map()
    ps = sorted(nuA[mA[i * 2 + k]] * nuB[mB[k * 2 + j]] for i in range(2) for k in range(2) for j in range(2))
    taus = np.array([ps[-1] * 1.01] + [ps[t] * 1.0000001 for t in range(7, -1, -1)] + [ps[0] * 0.5])
    bound = oracle.cse_tree(A, B, taus)
    for m, tau in enumerate(taus):
        tot = Fraction(0)
        for i in range(2):
            for j in range(2):
                s = Fraction(0)
                for k in range(2):
                    p = nuA[mA[i * 2 + k]] * nuB[mB[k * 2 + j]]
                    if p < tau:
                        s += Fraction(float(p))
                tot += s * s
        getcontext().prec = 60
        exact = float((Decimal(tot.numerator) / Decimal(tot.denominator)).sqrt())
        assert abs(bound[m] - exact) <= 8 * math.ulp(max(exact, 1e-300))


@pytest.mark.parametrize("nb,b,seed", [(3, 4, 0), (4, 2, 1), (5, 3, 2), (6, 2, 3), (8, 2, 4), (7, 4, 5)])
def test_bruteforce_and_orderings(nb, b, seed):
    rng = np.random.default_rng(seed)
    A = rand_bsm(rng, nb, b, 0.6, decay=0.7, zero_blocks=0.1)
    B = rand_bsm(rng, nb, b, 0.6, decay=0.7, zero_blocks=0.1, n=A.n)
    taus = synth.tau_log(24, -12.0) * 10.0
    bound = oracle.cse_tree(A, B, taus)
    flat, ssum = oracle.cse_flat_sum(A, B, taus)
    assert np.all(np.diff(bound) <= 0.0)                       # monotone in tau
    for m, tau in enumerate(taus):
        bu = bottom_up_bound(A, B, tau)
        assert abs(bound[m] - bu) <= 1e-15 * max(bu, 1e-300) * 8
        meas = dense_spamm_error(A, B, tau)
        assert meas <= flat[m] * (1 + 1e-12) + 1e-300
        assert flat[m] <= bound[m] * (1 + 1e-12) + 1e-300
        assert bound[m] <= ssum[m] * (1 + 1e-12) + 1e-300


def test_zero_and_all_skipped():
    rng = np.random.default_rng(9)
    A = rand_bsm(rng, 4, 3, 0.7)
    B = rand_bsm(rng, 4, 3, 0.7, n=A.n)
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(B)
    ps = [nuA[a] * nuB[c] for a in range(A.nblk) for c in range(B.nblk)]
    taus = np.array([max(ps) * 2.0, min(ps) * 0.5])
    bound = oracle.cse_tree(A, B, taus)
    normA = np.linalg.norm(A.to_dense()); normB = np.linalg.norm(B.to_dense())
    assert bound[0] <= normA * normB * (1 + 1e-12)            # everything skipped
    assert bound[0] >= np.linalg.norm(A.to_dense() @ B.to_dense()) * (1 - 1e-12)
    assert bound[1] == 0.0                                    # nothing skipped


def test_select_rule():
    taus = np.array([1.0, 0.1, 0.01, 0.001])
    bound = np.array([5.0, 0.2, 0.05, 0.0])
    assert oracle.select(bound, taus, 0.1) == (2, 0.01)
    assert oracle.select(bound, taus, 0.2) == (2, 0.01)      # strict <
    assert oracle.select(bound, taus, 0.2000001) == (1, 0.1)
    assert oracle.select(bound, taus, 0.0) == (4, 0.0)       # none -> exact product
    # brute force: the chosen bound is the largest one below the budget
    rng = np.random.default_rng(1)
    for _ in range(50):
        bd = np.sort(rng.random(10))[::-1]
        budget = rng.random()
        idx, tau = oracle.select(bd, np.linspace(1, 0.1, 10), budget)
        below = [m for m in range(10) if bd[m] < budget]
        if below:
            assert bd[idx] == max(bd[m] for m in below) and idx == min(below)
        else:
            assert idx == 10 and tau == 0.0


def test_paper_tau_list():
    fx = json.load(open(os.path.join(GOLD, "tau_list_section_eval.json")))
    t = synth.tau_paper(fx["N"])
    assert t.shape[0] == fx["N"] and t[0] == fx["first"]
    assert np.all(t[1:] < t[:-1])
    assert abs(math.log10(t[-1]) - fx["last_order_of_magnitude"]) < 0.5


# ---------------------------------------------------------------------------
# precision-tier mode of the bound (mixed-precision leaf products)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_tier_mode_special_cases(seed):
    rng = np.random.default_rng(300 + seed)
    A = rand_bsm(rng, 6, 3, 0.7, decay=0.8)
    B = rand_bsm(rng, 6, 3, 0.7, decay=0.8, n=A.n)
    taus = synth.tau_log(24, -12.0) * 10.0
    base = oracle.cse_tree(A, B, taus)
    for t0 in [taus[5], taus[12], 0.0]:
        b0 = oracle.cse_tree(A, B, np.array([t0 if t0 > 0 else 1e-300]))[0]
        # no low tier below tau0: every sigma <= tau0 gives the plain bound at tau0
        low = np.array([t for t in taus if t <= t0]) if t0 > 0 else np.array([1e-300])
        if low.size:
            m1 = oracle.cse_tree(A, B, low, mode=1, tau0=t0, c_low=0.3)
            assert np.all(m1 == b0)
        # c = 1: the tier costs as much as skipping, i.e. the plain bound at sigma
        hi = np.array([t for t in taus if t >= t0])
        m1 = oracle.cse_tree(A, B, hi, mode=1, tau0=t0, c_low=1.0)
        assert np.array_equal(m1, base[:hi.shape[0]])
        # c = 0: a free tier gives the plain bound at tau0 for every sigma
        m0 = oracle.cse_tree(A, B, hi, mode=1, tau0=t0, c_low=0.0)
        assert np.all(m0 == b0)


@pytest.mark.parametrize("b", [32, 64])
def test_fp32_tier_constant_bounds_fp32_products(b):
    """||fl32(A) fl32(B) (FP32 arithmetic) - AB||_F <= c_32 ||A||_F ||B||_F."""
    rng = np.random.default_rng(b)
    c = oracle.tier_constant(1, b)
    assert 3e-6 < c < 1e-5
    worst = 0.0
    for _ in range(200):
        A = rng.standard_normal((b, b)) * np.exp(rng.uniform(-20, 5))
        B = rng.standard_normal((b, b)) * np.exp(rng.uniform(-20, 5))
        if rng.random() < 0.3:
            A = np.abs(A); B = np.abs(B)            # no cancellation: the worst case for the bound
        P32 = (A.astype(np.float32) @ B.astype(np.float32)).astype(np.float64)
        err = np.linalg.norm(P32 - A @ B)
        ratio = err / (np.linalg.norm(A) * np.linalg.norm(B))
        worst = max(worst, ratio)
        assert ratio <= c
    assert worst > 1e-9                             # the FP32 path really rounded


def _rn_bf16(x):
    """Round to the nearest BF16 value (8 significant bits, ties to even,
    subnormal spacing 2^-133), exactly, in float64."""
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    q = np.maximum(e - 8, -133).astype(np.float64)
    return np.rint(np.ldexp(x, (-q).astype(np.int64))) * np.exp2(q)


@pytest.mark.parametrize("b", [32, 64])
def test_bf16x3_tier_constant_bounds_split_products(b):
    """||2^(ea+eb) (hi_a hi_b + hi_a lo_b + lo_a hi_b) (FP32) - AB||_F <=
    c_bf16 ||A||_F ||B||_F, with each block scaled by a power of two to a
    maximum in [1, 2) and split hi = RN_bf16(x), lo = RN_bf16(x - hi)."""
    rng = np.random.default_rng(100 + b)
    c = oracle.tier_constant(2, b)
    assert c > oracle.tier_constant(1, b) and c < 1e-4
    worst = 0.0
    for t in range(200):
        A = rng.standard_normal((b, b)) * np.exp(rng.uniform(-20, 5))
        B = rng.standard_normal((b, b)) * np.exp(rng.uniform(-20, 5))
        if t % 3 == 0:
            A = np.abs(A); B = np.abs(B)                        # no cancellation
        if t % 5 == 0:                                          # entries far below the BF16 range
            A[rng.random((b, b)) < 0.3] *= 1e-45
        parts = []
        for M in (A, B):
            e = np.frexp(np.max(np.abs(M)))[1]
            Ms = np.ldexp(M, 1 - e)                             # max in [1, 2)
            hi = _rn_bf16(Ms)
            lo = _rn_bf16(Ms - hi)
            parts.append((hi.astype(np.float32), lo.astype(np.float32), e - 1))
        (ah, al, ea), (bh, bl, eb) = parts
        S = (ah @ bh) + (ah @ bl) + (al @ bh)                   # FP32 arithmetic
        P = np.ldexp(S.astype(np.float64), ea + eb)
        err = np.linalg.norm(P - A @ B)
        ratio = err / (np.linalg.norm(A) * np.linalg.norm(B))
        worst = max(worst, ratio)
        assert ratio <= c
    assert worst > 1e-7                                         # the split really rounded


def test_bf16_rounding_helper():
    # exact values, ties to even, subnormal spacing
    assert _rn_bf16(1.0) == 1.0
    assert _rn_bf16(1.0 + 2.0 ** -9) == 1.0                     # below half a spacing (2^-7)
    assert _rn_bf16(1.0 + 2.0 ** -8) == 1.0                     # tie -> even (down)
    assert _rn_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie -> even (up)
    assert _rn_bf16(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    assert _rn_bf16(3 * 2.0 ** -134) == 2.0 ** -132             # subnormal spacing 2^-133, tie to even
    assert _rn_bf16(2.0 ** -140) == 0.0


@pytest.mark.parametrize("seed", range(3))
def test_leaf_bounds_tier_mode(seed):
    """Tier mode of B_flat / B_sum: the same special cases as the recursive
    bound's tier mode (sigma <= tau0 or c = 0: the plain bound at tau0;
    c = 1: the plain bound at sigma), and both bound the error of a product
    that skips p < tau0, evaluates tau0 <= p < sigma in FP32 (folded into
    FP64 per pair) and the rest in FP64, against the exact product."""
    rng = np.random.default_rng(400 + seed)
    A = rand_bsm(rng, 6, 8, 0.7, decay=0.8)
    B = rand_bsm(rng, 6, 8, 0.7, decay=0.8, n=A.n)
    taus = synth.tau_log(24, -12.0) * 10.0
    fl, sm = oracle.cse_flat_sum(A, B, taus)
    for t0 in [taus[5], taus[12]]:
        f0, s0 = oracle.cse_flat_sum(A, B, np.array([t0]))
        low = np.array([t for t in taus if t <= t0])
        f1, s1 = oracle.cse_flat_sum(A, B, low, mode=1, tau0=t0, c_low=0.3)
        assert np.all(f1 == f0[0]) and np.all(s1 == s0[0])
        hi = np.array([t for t in taus if t >= t0])
        f1, s1 = oracle.cse_flat_sum(A, B, hi, mode=1, tau0=t0, c_low=1.0)
        assert np.array_equal(f1, fl[:hi.shape[0]]) and np.array_equal(s1, sm[:hi.shape[0]])
        f1, s1 = oracle.cse_flat_sum(A, B, hi, mode=1, tau0=t0, c_low=0.0)
        assert np.all(f1 == f0[0]) and np.all(s1 == s0[0])
    # the bound holds for a real tiered product
    b = A.b
    c = oracle.tier_constant(1, b)
    nuA, nuB = oracle.norms(A)[1], oracle.norms(B)[1]
    exact = A.to_dense() @ B.to_dense()
    mA, mB = A.block_map(), B.block_map()
    nb = A.nb
    ps = np.array([nuA[mA[i * nb + k]] * nuB[mB[k * nb + j]] for i in range(nb) for k in range(nb)
                   for j in range(nb) if mA[i * nb + k] >= 0 and mB[k * nb + j] >= 0])
    for q0, q1 in [(0.2, 0.6), (0.5, 0.9)]:
        t0, sig = np.quantile(ps, q0), np.quantile(ps, q1)
        assert np.sum(ps < t0) > 0 and np.sum((ps >= t0) & (ps < sig)) > 0
        C = np.zeros((nb * b, nb * b))
        for i in range(nb):
            for j in range(nb):
                acc = np.zeros((b, b))
                for k in range(nb):
                    sa, sb = mA[i * nb + k], mB[k * nb + j]
                    if sa < 0 or sb < 0:
                        continue
                    p = nuA[sa] * nuB[sb]
                    Ab, Bb = A.vals[sa].T, B.vals[sb].T
                    if p < t0:
                        continue
                    if p < sig:
                        acc = acc + (Ab.astype(np.float32) @ Bb.astype(np.float32)).astype(np.float64)
                    else:
                        acc = acc + Ab @ Bb
                C[i * b:(i + 1) * b, j * b:(j + 1) * b] = acc
        err = np.linalg.norm(C[:A.n, :A.n] - exact)
        f1, s1 = oracle.cse_flat_sum(A, B, np.array([sig]), mode=1, tau0=t0, c_low=c)
        tr = oracle.cse_tree(A, B, np.array([sig]), mode=1, tau0=t0, c_low=c)
        # (the FP64 pairs' own rounding, ~1e-16 of the product, is outside the bound)
        assert err <= f1[0] + 1e-13 * np.linalg.norm(exact)
        assert f1[0] <= tr[0] * (1 + 1e-12) and tr[0] <= s1[0] * (1 + 1e-12)
        assert f1[0] > 0
