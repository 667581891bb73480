"""Adversarial pins of the oracle's constants and rules (CPU only).

Each test builds the case where one term of a rule is what keeps it
correct, so that dropping or weakening that term fails it:

* the split-BF16 tier constant: a block at the worst split point, with the
  FP32 accumulation rounding the same way as the dropped terms, reaches more
  than half of c_bf16; its representation part is reached by the dropped
  terms alone (exact arithmetic), its accumulation part by 3b additions
  under the error model the constant assumes (unit roundoff 2^-23 each);
* the truncation: a key sum that lands exactly on floor(T/Q) with
  T = RN(delta^2) rounded up must not be removed (the strict <), and the
  removal is maximal up to the key quantum;
* the tolerance schedule: the Davis-Kahan sum of the perturbations spends
  eps/2 over n_max + 1 of them, stays below eps/2 along recorded runs, and
  the result is within eps of the exact projector;
* the stop rule: never fires on exact-arithmetic (dense FP64) SP2 runs
  before the rounding floor, and fires soon after a perturbed run reaches
  its floor.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


# ---------------------------------------------------------------------------
# helpers: exact roundings
# ---------------------------------------------------------------------------

def _rn_bf16(x: float) -> float:
    """Round a double to the nearest BF16 value (8 significant bits, ties to
    even; normal range only, which is all these tests use)."""
    m, e = math.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    q = e - 8
    return float(round(Fraction(x) / Fraction(2) ** q) * Fraction(2) ** q)


def _rd_fp32(v: Fraction) -> Fraction:
    """The largest FP32 value <= v (round toward -inf), for 0 < v < 2^100."""
    assert v > 0
    e = v.numerator.bit_length() - v.denominator.bit_length()
    if Fraction(2) ** e > v:
        e -= 1                                # 2^e <= v < 2^(e+1)
    ulp = Fraction(2) ** (e - 23)
    return math.floor(v / ulp) * ulp


def _split(x: float):
    hi = _rn_bf16(x)
    lo = _rn_bf16(x - hi)
    return hi, lo


# the worst split point in [1, 2): hi = 1 + 2^-7, x - hi just below 2^-8 so
# that lo = RN_bf16(x - hi) = 255 * 2^-16 and the residual x - hi - lo is just
# below half of lo's spacing (2^-17); hi * lo then ends in six 1 bits below
# the FP32 spacing of the accumulator (2^-17 at 64, 2^-18 at 32)
_HI = 1.0 + 2.0 ** -7
_LO = 255.0 * 2.0 ** -16
_X = _HI + _LO + (2.0 ** -17 - 2.0 ** -30)


def _split_terms_all_equal(b: int):
    """The exact products an output entry of A B accumulates in the
    split-BF16 tier when every entry of A and B equals _X: b of hi*hi, then b
    of hi*lo, then b of lo*hi (the three MFMA passes)."""
    hi, lo = _split(_X)
    assert (hi, lo) == (_HI, _LO)
    H, L = Fraction(hi), Fraction(lo)
    return [H * H] * b + [H * L] * b + [L * H] * b


@pytest.mark.parametrize("b", [32, 64])
def test_bf16x3_constant_reaches_worst_split_case(b):
    """All-equal blocks at the worst split point, accumulated in FP32 with
    rounding toward -inf (a rounding the constant's unit roundoff 2^-23
    covers) in the three-pass order: the dropped terms and the accumulation
    both push the result down, and the error reaches more than half of
    c_bf16 ||A||_F ||B||_F (so dropping the representation term kappa from
    the constant fails here)."""
    terms = _split_terms_all_equal(b)
    acc = Fraction(0)
    for t in terms:
        acc = _rd_fp32(acc + t)
    x = Fraction(_X)
    exact = b * x * x                          # every entry of A B
    # every entry has the same error, and ||A||_F ||B||_F = b^2 x^2, so the
    # block ratio ||fl(AB) - AB||_F / (||A||_F ||B||_F) is the entry ratio
    ratio = float((exact - acc) / (b * x * x))
    c = oracle.tier_constant(2, b)
    assert ratio <= c
    assert ratio >= 0.5 * c, (ratio, c)


@pytest.mark.parametrize("b", [32, 64])
def test_bf16x3_representation_part(b):
    """Exact arithmetic on the split operands: the dropped terms alone
    (lo*lo and the split residuals) reach more than half of the constant's
    representation part at the worst split point, and stay below it on
    random, all-positive and worst-point blocks."""
    parts = oracle.tier_constant_parts(2, b)
    kappa = parts["represent"]
    x = Fraction(_X)
    H, L = Fraction(_HI), Fraction(_LO)
    worst = float((x * x - H * H - 2 * H * L) / (x * x))
    assert 0.5 * kappa <= worst <= kappa, (worst, kappa)
    rng = np.random.default_rng(7 + b)
    for t in range(40):
        A = rng.standard_normal((b, b))
        B = rng.standard_normal((b, b))
        if t % 2:
            A, B = np.abs(A), np.abs(B)
        terms_err = 0.0
        As = np.ldexp(A, 1 - np.frexp(np.max(np.abs(A)))[1])
        Bs = np.ldexp(B, 1 - np.frexp(np.max(np.abs(B)))[1])
        ah = np.vectorize(_rn_bf16)(As)
        al = np.vectorize(_rn_bf16)(As - ah)
        bh = np.vectorize(_rn_bf16)(Bs)
        bl = np.vectorize(_rn_bf16)(Bs - bh)
        # products of 8-bit values summed in FP64: exact to ~2^-50 relative
        S = ah @ bh + ah @ bl + al @ bh
        terms_err = np.linalg.norm(S - As @ Bs) / (np.linalg.norm(As) * np.linalg.norm(Bs))
        assert terms_err <= kappa


@pytest.mark.parametrize("precision,b", [(1, 32), (1, 64), (2, 32), (2, 64)])
def test_accumulation_part_covers_every_addition(precision, b):
    """Under the error model the tier constants assume (each FP32 addition
    returns (s + t)(1 + d), |d| <= 2^-23, in an order the hardware does not
    document), an output entry whose first product dominates loses about
    2^-23 of it at every later addition.  The FP32 tier adds b products per
    entry, the split-BF16 tier 3b (hi*hi, hi*lo, lo*hi): the accumulation
    part must cover all of them (a gamma_b in place of gamma_3b fails)."""
    parts = oracle.tier_constant_parts(precision, b)
    # one row of A times one column of B: a_0 = c_0 dominates, the other
    # entries are small but nonzero, with nonzero low parts
    a = [1.0 + 2.0 ** -7 + 2.0 ** -12] + [2.0 ** -12 * (1.0 + 2.0 ** -7 + 2.0 ** -12)] * (b - 1)
    if precision == 1:
        terms = [Fraction(float(np.float32(v))) ** 2 for v in a]
    else:
        sp = [_split(v) for v in a]
        assert all(lo != 0.0 for _, lo in sp)
        terms = ([Fraction(h) * Fraction(h) for h, _ in sp] + [Fraction(h) * Fraction(lo) for h, lo in sp]
                 + [Fraction(lo) * Fraction(h) for h, lo in sp])
    assert len(terms) == (b if precision == 1 else 3 * b)
    ud = Fraction(1, 2 ** 23)
    s = terms[0]
    for t in terms[1:]:
        s = (s + t) * (1 - ud)                 # the model's adversarial rounding
    exact = sum(terms, Fraction(0))
    norm_ab = sum((Fraction(float(np.float32(v)) if precision == 1 else v) ** 2 for v in a), Fraction(0))
    ratio = float((exact - s) / norm_ab)       # ||A||_F ||B||_F = ||a||^2 (rank one)
    acc = parts["accumulate"]
    assert ratio <= acc
    assert ratio >= 0.9 * acc, (ratio, acc)


@pytest.mark.parametrize("precision,b", [(1, 32), (1, 64), (2, 32), (2, 64)])
def test_tier_constant_is_its_parts(precision, b):
    p = oracle.tier_constant_parts(precision, b)
    total = (p["represent"] + p["accumulate"] + p["underflow"]) * (1.0 + 2.0 ** -40)
    assert oracle.tier_constant(precision, b) == total


# ---------------------------------------------------------------------------
# truncation
# ---------------------------------------------------------------------------

def _four_squares(k: int):
    """Four non-negative integers whose squares sum to k (Lagrange)."""
    a = math.isqrt(k)
    while a >= 0:
        r = k - a * a
        bb = math.isqrt(r)
        for b_ in range(bb, max(-1, bb - 64), -1):
            r2 = r - b_ * b_
            c = math.isqrt(r2)
            while c >= 0 and 2 * c * c >= r2:
                d2 = r2 - c * c
                d = math.isqrt(d2)
                if d * d == d2:
                    return a, b_, c, d
                c -= 1
        a -= 1
    raise AssertionError("no decomposition")


def _delta_rounding_up_onto_grid():
    """A delta in [1, sqrt 2) whose square rounds UP to T = RN(delta^2) with
    T on the key grid (T / Q an integer, Q = 2^-40)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        cand = 1.0 + rng.random(200000) * 0.4
        T = cand * cand
        mant = (T.view(np.uint64) & np.uint64((1 << 52) - 1))
        ok = np.nonzero((mant & np.uint64(0xFFF)) == 0)[0]
        for i in ok:
            d = float(cand[i])
            if Fraction(d) ** 2 < Fraction(float(T[i])):
                return d
    raise AssertionError("no delta found")


def _diag_units(nb, b, keys_scaled):
    """A block-diagonal matrix whose diagonal block r holds four entries
    m * 2^-20 with sum of m^2 = keys_scaled[r]: its exact sum of squares is
    keys_scaled[r] * 2^-40, exactly representable."""
    vals = np.zeros((nb, b, b))
    for r, k in enumerate(keys_scaled):
        for j, m in enumerate(_four_squares(int(k))):
            vals[r, j, j] = m * 2.0 ** -20
    idx = np.arange(nb, dtype=np.int32)
    return oracle.BSM(nb * b, b, idx, idx.copy(), vals)


def _exact_sq(X, keep):
    return sum((Fraction(float(v)) ** 2 for v in np.ravel(X.vals[keep])), Fraction(0))


def test_truncation_key_sum_on_the_budget_is_kept():
    """T = RN(delta^2) rounded up and lies on the key grid; units A and B
    have exact sums of squares Q kA, Q kB with kA + kB = floor(T/Q) = K_T.
    Removing both would give ||E||_F^2 = T > delta^2, so the rule's strict
    < must keep B: a <= (searchsorted side 'right') fails here."""
    delta = _delta_rounding_up_onto_grid()
    T, Q = delta * delta, 2.0 ** -40           # T in [1, 2): the key quantum is 2^-40
    kt = int(Fraction(T) / Fraction(Q))
    assert Fraction(T) == kt * Fraction(Q) and Fraction(delta) ** 2 < Fraction(T)
    kA = kt // 3
    kB = kt - kA
    X = _diag_units(3, 32, [kA, kB, 4 * kt])
    sq, _ = oracle.norms(X)
    assert [Fraction(float(v)) for v in sq[:2]] == [Q * kA, Q * kB]   # sq exact, keys exact
    Xt, info = oracle.truncate(X, delta)
    removed = ~np.isin(X.keys(), Xt.keys())
    assert list(np.nonzero(removed)[0]) == [0]
    assert _exact_sq(X, removed) < Fraction(delta) ** 2
    # the construction really sits on the boundary: A and B together break it
    both = np.array([True, True, False])
    assert _exact_sq(X, both) >= Fraction(delta) ** 2


@pytest.mark.parametrize("gap_keys", [1, 2, 4096, 10 ** 6])
def test_truncation_is_maximal_within_the_key_quantum(gap_keys):
    """Units A and B with kA + kB = K_T - gap_keys fit below the budget, so
    both must go (a budget kept back from K_T by a margin of ~2^-29 T would
    keep B); generally, the first unit the rule keeps could not have been
    removed: the exact removed sum with it is at least
    delta^2 (1 - 2^-51) - (q + 2) Q."""
    delta = _delta_rounding_up_onto_grid() * 1.001
    T, Q = delta * delta, 2.0 ** -40
    assert 1.0 <= T < 2.0
    kt = math.floor(Fraction(T) / Fraction(Q))
    kA = kt // 3
    kB = kt - kA - gap_keys
    X = _diag_units(3, 32, [kA, kB, 4 * kt])
    Xt, info = oracle.truncate(X, delta)
    removed = ~np.isin(X.keys(), Xt.keys())
    assert list(np.nonzero(removed)[0]) == [0, 1]
    assert _exact_sq(X, removed) < Fraction(delta) ** 2
    # generic maximality on random symmetric matrices as well
    rng = np.random.default_rng(gap_keys % 1000)
    nb, b = 6, 32
    Y = _diag_units(nb, b, list(rng.integers(1 << 30, 1 << 36, nb)))
    sqY, _ = oracle.norms(Y)
    tot = float(np.sum(sqY))
    for frac in (0.1, 0.37, 0.9):
        dl = math.sqrt(tot * frac)
        Yt, inf = oracle.truncate(Y, dl)
        rem = ~np.isin(Y.keys(), Yt.keys())
        q = int(np.sum(rem))
        kept_idx = np.argsort(sqY + rem * 1e300)[0] if q < nb else None
        if kept_idx is not None:
            Q2 = math.ldexp(1.0, math.frexp(dl * dl)[1] - 1 - 40)
            with_next = rem.copy()
            with_next[kept_idx] = True
            lhs = _exact_sq(Y, with_next)
            rhs = Fraction(dl) ** 2 * (1 - Fraction(1, 2 ** 51)) - (q + 2) * Fraction(Q2)
            assert lhs >= rhs


# ---------------------------------------------------------------------------
# tolerance schedule and stop rule
# ---------------------------------------------------------------------------

def test_schedule_spends_half_the_tolerance_over_n_max_steps():
    """sum over the n_max + 1 perturbations (X~_0 and n_max steps) of the
    Davis-Kahan drift sqrt(2) delta_i / g_i is eps / 2 for any gaps."""
    rng = np.random.default_rng(5)
    for n_max in (20, 60, 100):
        p = oracle.SP2Params(n_occ=1, eps=1e-6, n_max=n_max)
        gaps = np.exp(rng.uniform(math.log(1e-3), 0.0, n_max + 1))
        s = math.fsum(math.sqrt(2.0) * oracle.step_delta(p, g) / g for g in gaps)
        assert abs(s - p.eps / 2) <= 1e-12 * p.eps


def _gersch(F):
    r = np.sum(np.abs(F), 1) - np.abs(np.diag(F))
    return float(np.min(np.diag(F) - r)), float(np.max(np.diag(F) + r))


@pytest.mark.parametrize("which", ["chain", "3d"])
def test_schedule_error_sum_along_recorded_runs(which):
    """Along a recorded hybrid run: the mapped gaps g_i (from the exact
    HOMO/LUMO through the recorded branches) give sum sqrt(2) delta_i / g_i
    <= eps/2; with the distance of the result from its own projector,
    2 |e_final|, the a-posteriori estimate is below eps, and the result is
    within eps of the exact projector."""
    if which == "chain":
        Fm, n_occ, taus = synth.chain1d(512, 1, 32), 256, synth.tau_paper()
    else:
        Fm, n_occ, taus = synth.sys3d(768, 2, 32), 384, synth.tau_log(32)
    F = oracle.BSM.of(Fm)
    Fd = F.to_dense()
    w, U = np.linalg.eigh(Fd)
    D = U[:, :n_occ] @ U[:, :n_occ].T
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, homo=w[n_occ - 1], lumo=w[n_occ])
    Dt, logs, info = oracle.sp2(F, p)
    lmin, lmax = _gersch(Fd)
    W = lmax - lmin
    xh, xl = (lmax - w[n_occ - 1]) / W, (lmax - w[n_occ]) / W
    drift = math.sqrt(2.0) * info["delta0"] / (xh - xl)         # delta_0
    for lg in logs:
        if lg.branch < 0:
            break
        xh, xl = (xh * xh, xl * xl) if lg.branch == 0 else (2 * xh - xh * xh, 2 * xl - xl * xl)
        drift += math.sqrt(2.0) * lg.delta / (xh - xl)
    assert drift <= p.eps / 2 * (1 + 1e-9)
    assert drift + 2 * abs(logs[-1].e) < p.eps
    assert np.linalg.norm(Dt.to_dense() - D) < p.eps


def _dense_sp2_e(F, n_occ, n_steps, noise=0.0, seed=0):
    """e_i = tr X_i - ||X_i||_F^2 of dense FP64 SP2 (trace-closest branch),
    optionally with a symmetric perturbation of Frobenius norm `noise` added
    after every step."""
    rng = np.random.default_rng(seed)
    lmin, lmax = _gersch(F)
    n = F.shape[0]
    X = (lmax * np.eye(n) - F) / (lmax - lmin)
    es = []
    for _ in range(n_steps):
        t1 = np.trace(X)
        X2 = X @ X
        es.append(t1 - float(np.sum(X * X)))
        X = X2 if abs(np.trace(X2) - n_occ) <= abs(2 * t1 - np.trace(X2) - n_occ) else 2 * X - X2
        if noise:
            E = rng.standard_normal((n, n))
            E = E + E.T
            X = X + E * (noise / np.linalg.norm(E))
    return es


@pytest.mark.parametrize("which", ["chain", "3d"])
def test_stop_rule_silent_on_exact_sp2(which):
    """Dense FP64 SP2 (no SpAMM, no truncation): the rule stays silent while
    e is above the rounding floor (|e| > 1e-9) and fires within three steps
    of e reaching it."""
    if which == "chain":
        F, n_occ = oracle.BSM.of(synth.chain1d(512, 1, 32)).to_dense(), 256
    else:
        F, n_occ = oracle.BSM.of(synth.sys3d(768, 2, 32)).to_dense(), 384
    es = _dense_sp2_e(F, n_occ, 70)
    fired = next(i for i in range(1, len(es) + 1) if oracle.should_stop(es[:i], 0.0))
    first_floor = next(i for i, e in enumerate(es) if abs(e) <= 1e-9)
    assert all(abs(e) > 1e-9 for e in es[:fired - 1][:first_floor])
    assert first_floor <= fired - 1 <= first_floor + 3, (first_floor, fired, es[first_floor - 2:fired])


def test_stop_rule_fires_at_a_perturbation_floor():
    """Dense SP2 with a perturbation of norm 1e-7 after every step: e stalls
    near the floor the perturbations set, and the rule stops the run within
    three steps of e first falling below 1e-5 instead of running on."""
    F, n_occ = oracle.BSM.of(synth.sys3d(768, 2, 32)).to_dense(), 384
    es = _dense_sp2_e(F, n_occ, 70, noise=1e-7, seed=3)
    fired = next(i for i in range(1, len(es) + 1) if oracle.should_stop(es[:i], 0.0))
    first = next(i for i, e in enumerate(es) if abs(e) <= 1e-5)
    assert fired - 1 <= first + 3, (first, fired, es[first - 2:fired])
    assert all(abs(e) > 1e-5 for e in es[:first])


# ---------------------------------------------------------------------------
# leaf-level bounds: exactly rounded sums over the outputs
# ---------------------------------------------------------------------------

def _diag_single(nb, b, values):
    """Block-diagonal matrix whose block (i, i) holds values[i] at its first
    entry: nu(block i) = |values[i]| exactly."""
    vals = np.zeros((nb, b, b))
    vals[:, 0, 0] = values
    idx = np.arange(nb, dtype=np.int32)
    return oracle.BSM(nb * b, b, idx, idx.copy(), vals)


def test_leaf_bounds_round_the_output_sum_once():
    """Outputs whose skipped products are 1, 2^-53, 2^-53: the exact sum
    1 + 2^-52 rounds to itself, while adding the outputs one after another
    in double would stop at 1 (each addition a tie to even).  Likewise for
    B_flat with one term 1 and 32 terms 2^-56: the exact sum 1 + 2^-51 gives
    sqrt_RN = 1 + 2^-52, the running sum stays at 1."""
    b = 32
    A = _diag_single(3, b, [1.0, 2.0 ** -26, 2.0 ** -26])
    B = _diag_single(3, b, [1.0, 2.0 ** -27, 2.0 ** -27])
    flat, ssum = oracle.cse_flat_sum(A, B, np.array([4.0]))
    assert ssum[0] == 1.0 + 2.0 ** -52
    seq = 0.0
    for v in (1.0, 2.0 ** -53, 2.0 ** -53):
        seq += v
    assert seq == 1.0                       # the order-dependent running sum differs
    A = _diag_single(33, b, [1.0] + [2.0 ** -14] * 32)
    B = _diag_single(33, b, [1.0] + [2.0 ** -14] * 32)
    flat, ssum = oracle.cse_flat_sum(A, B, np.array([4.0]))
    exact = Fraction(1) + 32 * Fraction(2) ** -56
    assert Fraction(float(exact)) == exact
    assert flat[0] == math.sqrt(float(exact)) == 1.0 + 2.0 ** -52
    # a sum that is exactly a tie rounds to even
    A = _diag_single(2, b, [1.0, 2.0 ** -26])
    B = _diag_single(2, b, [1.0, 2.0 ** -27])
    flat, ssum = oracle.cse_flat_sum(A, B, np.array([4.0]))
    assert ssum[0] == 1.0


@pytest.mark.parametrize("seed", range(3))
def test_leaf_bounds_equal_exact_rational_sums(seed):
    """On random block-sparse inputs the bounds equal sums evaluated with
    exact rationals from the per-output k-ascending double sums."""
    rng = np.random.default_rng(900 + seed)
    nb, b = 5, 32
    def rnd():
        keep = rng.random((nb, nb)) < 0.6
        rr, cc = np.nonzero(keep)
        vals = np.zeros((rr.shape[0], b, b))
        vals[:, 0, 0] = np.exp(rng.uniform(-20, 2, rr.shape[0]))
        vals[:, 1, 3] = np.exp(rng.uniform(-30, 0, rr.shape[0]))
        return oracle.BSM(nb * b, b, rr.astype(np.int32), cc.astype(np.int32), vals)
    A, B = rnd(), rnd()
    nuA, nuB = oracle.norms(A)[1], oracle.norms(B)[1]
    mA, mB = A.block_map(), B.block_map()
    taus = synth.tau_log(12, -12.0)
    flat, ssum = oracle.cse_flat_sum(A, B, taus, nuA, nuB)
    for m, t in enumerate(taus):
        S, F2 = Fraction(0), Fraction(0)
        for i in range(nb):
            for j in range(nb):
                s = 0.0
                for k in range(nb):
                    sa, sb = mA[i * nb + k], mB[k * nb + j]
                    if sa < 0 or sb < 0:
                        continue
                    p = nuA[sa] * nuB[sb]
                    if p < t:
                        s += p
                S += Fraction(s)
                F2 += Fraction(s * s)
        assert ssum[m] == float(S)
        assert flat[m] == math.sqrt(float(F2))


# ---------------------------------------------------------------------------
# the FP32 tier's operand-norm guard
# ---------------------------------------------------------------------------

def _ftz32(x):
    """Round to FP32 and flush values below the normal range to zero (the
    worst a flush-to-zero datapath does)."""
    y = np.asarray(x, dtype=np.float32).astype(np.float64)
    y[np.abs(y) < 2.0 ** -126] = 0.0
    return y


@pytest.mark.parametrize("b", [32, 64])
def test_fp32_tier_guard_and_underflow_term(b):
    """A block whose entries all lie below FP32's normal range loses them
    entirely under flush-to-zero, an error of the whole product that no
    relative rounding constant covers: the FP32 tier must not take it, and
    oracle.low_tier_pairs keeps such pairs in FP64.  Blocks that pass the
    guard (norm >= 2^-40) but hold entries below 2^-126 stay within c_32,
    whose underflow term covers the flushed part."""
    rng = np.random.default_rng(b + 5)
    c = oracle.tier_constant(1, b)
    # below the guard: every entry subnormal in FP32
    A = rng.standard_normal((b, b)) * 2.0 ** -140
    B = rng.standard_normal((b, b))
    err = np.linalg.norm(_ftz32(A) @ _ftz32(B) - A @ B) / (np.linalg.norm(A) * np.linalg.norm(B))
    assert np.linalg.norm(A) < oracle.FP32_TIER_NORM_MIN and err > 1e-2 > 100 * c
    # at the guard: norm 2^-40, a third of the entries far below 2^-126
    for _ in range(20):
        A = rng.standard_normal((b, b))
        A[rng.random((b, b)) < 0.33] *= 2.0 ** -110
        A *= oracle.FP32_TIER_NORM_MIN / np.linalg.norm(A)
        B = rng.standard_normal((b, b))
        B *= oracle.FP32_TIER_NORM_MIN / np.linalg.norm(B) * 4.0
        P32 = (_ftz32(A).astype(np.float32) @ _ftz32(B).astype(np.float32)).astype(np.float64)
        err = np.linalg.norm(P32 - A @ B) / (np.linalg.norm(A) * np.linalg.norm(B))
        assert err <= c
    # the tier split: a pair with a block below the guard stays FP64
    nb = 3
    vals = np.zeros((nb, b, b))
    vals[0, 0, 0] = 1.0
    vals[1, 0, 0] = 2.0 ** -50              # below the guard
    vals[2, 0, 0] = 2.0 ** -20
    idx = np.arange(nb, dtype=np.int32)
    X = oracle.BSM(nb * b, b, np.concatenate([idx, [0, 1]]).astype(np.int32),
                   np.concatenate([idx, [1, 0]]).astype(np.int32),
                   np.concatenate([vals, vals[2:3], vals[2:3]]))
    X = X.sorted()
    nu = oracle.norms(X)[1]
    all_low = oracle.low_tier_pairs(X, 0.0, 1e300, nu, 2)      # split BF16: no guard
    fp32_low = oracle.low_tier_pairs(X, 0.0, 1e300, nu, 1)
    K = oracle.kept(X, X, 0.0, True, nu, nu)
    assert all_low == K.npairs and fp32_low < all_low
