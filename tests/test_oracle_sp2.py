"""Pins of the oracle's purification (Algorithms 1, 4 and 5 with SP2
polynomials):

* diagonal F -> the exact step function, tr(D) = N_occ exactly;
* chain and 3D systems -> ||D~ - D||_F < eps against dense eigh;
* zero tolerances reproduce plain dense SP2;
* per step: ||X^_i - f_i(X~_{i-1})||_F < delta_i/2 and ||E_i||_F < delta_i/2
  (the two conditions of Algorithm 5), delta_i for Algorithms 1 and 4."""
import numpy as np
import pytest

import oracle
import synth


def eigh_density(F, n_occ):
    w, U = np.linalg.eigh(F.to_dense())
    return U[:, :n_occ] @ U[:, :n_occ].T, w


def test_diagonal_f_exact_step():
    n, b = 96, 8
    rng = np.random.default_rng(0)
    f = rng.uniform(-2.0, 2.0, n)
    f[np.abs(f) < 0.3] += 0.6                                 # keep away from mu = 0
    n_occ = int(np.sum(f < 0.0))
    F = oracle.from_dense(np.diag(f), b)
    fs = np.sort(f)
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=synth.tau_paper(), homo=fs[n_occ - 1], lumo=fs[n_occ])
    D, logs, info = oracle.sp2(F, p)
    Dd = D.to_dense()
    want = np.diag((f < 0.0).astype(np.float64))
    assert np.array_equal(Dd, want)
    assert np.trace(Dd) == n_occ


def test_chain_vs_eigh():
    Fm = synth.chain1d(1024, 1, 32)
    F = oracle.BSM.of(Fm)
    Dref, w = eigh_density(F, 512)
    p = oracle.SP2Params(n_occ=512, eps=1e-6, taus=synth.tau_paper(), homo=w[511], lumo=w[512])
    D, logs, info = oracle.sp2(F, p)
    assert np.linalg.norm(D.to_dense() - Dref) < 1e-6
    assert 5 <= len(logs) <= 40


def test_sys3d_vs_eigh_and_step_conditions():
    n, b = 768, 32
    F = oracle.BSM.of(synth.sys3d(n, 7, b))
    n_occ = n // 2
    Dref, w = eigh_density(F, n_occ)
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=synth.tau_log(32), homo=w[n_occ - 1], lumo=w[n_occ])
    X, X0, st, _ = oracle.sp2_start(F, p)
    checked = 0
    while True:
        Xn, Xh, log, st = oracle.sp2_step(X, st, p)
        if Xn is None:
            break
        Xd = X.to_dense()
        f = Xd @ Xd if log.branch == 0 else 2 * Xd - Xd @ Xd
        assert np.linalg.norm(Xh.to_dense() - f) < log.delta / 2       # SpAMM error
        assert np.linalg.norm(Xn.to_dense() - Xh.to_dense()) < log.delta / 2  # truncation
        X = Xn
        checked += 1
    assert checked >= 10
    assert np.linalg.norm(X.to_dense() - Dref) < 1e-6


def test_zero_tolerance_is_dense_sp2():
    Fm = synth.chain1d(256, 3, 32)
    F = oracle.BSM.of(Fm)
    _, w = eigh_density(F, 128)
    p = oracle.SP2Params(n_occ=128, eps=1e-6, taus=synth.tau_paper(), homo=w[127], lumo=w[128],
                         delta_const=0.0, n_max=25)
    D, logs, info = oracle.sp2(F, p)
    assert all(l.tau == 0.0 for l in logs if l.branch >= 0)
    # plain dense SP2 with the same branch sequence
    lmin, lmax = info["lmin"], info["lmax"]
    X = (lmax * np.eye(F.n) - F.to_dense()) / (lmax - lmin)
    for l in logs:
        if l.branch < 0:
            break
        X = X @ X if l.branch == 0 else 2 * X - X @ X
    assert np.linalg.norm(D.to_dense() - X) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("variant", ["spamm", "truncmul"])
def test_other_variants_step_conditions(variant):
    n, b = 512, 32
    F = oracle.BSM.of(synth.sys3d(n, 8, b))
    n_occ = n // 2
    Dref, w = eigh_density(F, n_occ)
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=synth.tau_log(32), homo=w[n_occ - 1],
                         lumo=w[n_occ], variant=variant)
    X, X0, st, _ = oracle.sp2_start(F, p)
    while True:
        Xn, Xh, log, st = oracle.sp2_step(X, st, p)
        if Xn is None:
            break
        Xd = X.to_dense()
        f = Xd @ Xd if log.branch == 0 else 2 * Xd - Xd @ Xd
        assert np.linalg.norm(Xn.to_dense() - f) < log.delta            # whole step error
        if variant == "truncmul":
            assert log.tau == 0.0
        X = Xn
    assert np.linalg.norm(X.to_dense() - Dref) < 1e-6


@pytest.mark.parametrize("precision", [1, 2])
def test_tier_selection_converges(precision):
    """The tiered selection (tau from half the budget, then the largest sigma
    whose Algorithm 3 bound with folded c p terms fits the budget; c of the
    FP32 or the split-BF16 tier) keeps every step within delta/2 (the
    oracle's products are FP64, so this checks the budget split) and
    converges."""
    n = 768
    F = oracle.BSM.of(synth.sys3d(n, 7, 32))
    Dref, w = eigh_density(F, n // 2)
    p = oracle.SP2Params(n_occ=n // 2, eps=1e-6, taus=synth.tau_log(32), homo=w[n // 2 - 1], lumo=w[n // 2],
                         precision=precision)
    D, logs, info = oracle.sp2(F, p)
    steps = [l for l in logs if l.branch >= 0]
    assert any(l.npairs_low > 0 for l in steps)
    assert all(l.sigma == 0.0 or l.sigma > l.tau for l in steps if l.npairs_low > 0)
    assert np.linalg.norm(D.to_dense() - Dref) < 1e-6


@pytest.mark.parametrize("bound", ["flat", "sum"])
def test_leaf_bounds_step_conditions(bound):
    """Selection with the leaf-level bounds (eq. (6) at the leaves, or the
    plain sum of skipped products): both still bound the product error, so
    both Algorithm 5 conditions hold at every step and the run converges;
    on the same iterate, B_flat <= B_tree <= B_sum orders the selected
    indices idx_flat <= idx_tree <= idx_sum (a smaller bound admits a larger
    threshold)."""
    n, b = 768, 32
    F = oracle.BSM.of(synth.sys3d(n, 7, b))
    n_occ = n // 2
    Dref, w = eigh_density(F, n_occ)
    taus = synth.tau_log(32)
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, homo=w[n_occ - 1], lumo=w[n_occ], bound=bound)
    X, X0, st, _ = oracle.sp2_start(F, p)
    strict = 0
    while True:
        Xn, Xh, log, st = oracle.sp2_step(X, st, p)
        if Xn is None:
            break
        Xd = X.to_dense()
        f = Xd @ Xd if log.branch == 0 else 2 * Xd - Xd @ Xd
        assert np.linalg.norm(Xh.to_dense() - f) < log.delta / 2
        assert np.linalg.norm(Xn.to_dense() - Xh.to_dense()) < log.delta / 2
        nu = oracle.norms(X)[1]
        tree = oracle.cse_tree(X, X, taus, nu, nu)
        flat, ssum = oracle.cse_flat_sum(X, X, taus, nu, nu)
        assert np.array_equal(log.bound, flat if bound == "flat" else ssum)
        i_tree = oracle.select(tree, taus, log.delta / 2)[0]
        i_flat = oracle.select(flat, taus, log.delta / 2)[0]
        i_sum = oracle.select(ssum, taus, log.delta / 2)[0]
        assert i_flat <= i_tree <= i_sum
        assert log.idx == (i_flat if bound == "flat" else i_sum)
        strict += int(i_flat < i_sum)
        X = Xn
    assert strict > 0
    assert np.linalg.norm(X.to_dense() - Dref) < 1e-6


@pytest.mark.parametrize("precision", [1, 2])
def test_leaf_bound_tier_selection_converges(precision):
    """The tier selection with B_flat (tau from a share of the budget, then
    sigma from the tier mode of B_flat) uses low-tier pairs and converges;
    at every step sigma's B_flat is below the product budget."""
    n = 768
    F = oracle.BSM.of(synth.sys3d(n, 7, 32))
    Dref, w = eigh_density(F, n // 2)
    taus = synth.tau_log(32)
    p = oracle.SP2Params(n_occ=n // 2, eps=1e-6, taus=taus, homo=w[n // 2 - 1], lumo=w[n // 2],
                         precision=precision, bound="flat")
    X, X0, st, _ = oracle.sp2_start(F, p)
    c = oracle.tier_constant(precision, 32)
    nlow = 0
    while True:
        Xn, Xh, log, st = oracle.sp2_step(X, st, p)
        if Xn is None:
            break
        if log.sidx < len(taus):
            nu = oracle.norms(X)[1]
            f2, _ = oracle.cse_flat_sum(X, X, np.array([log.sigma]), nu, nu, mode=1, tau0=log.tau, c_low=c)
            assert f2[0] < log.delta / 2
        nlow += log.npairs_low
        X = Xn
    assert nlow > 0
    assert np.linalg.norm(X.to_dense() - Dref) < 1e-6


def test_stop_rule_cases():
    """The stop rule on explicit histories (oldest first): e_tol, and the
    quadratic-convergence test |e_i| > 4 e_{i-2}^2 / (1 - 2|e_{i-2}|)^2,
    applied once |e_{i-2}| <= 1/8."""
    S = oracle.should_stop
    assert not S([], 0.0)
    assert S([0.5, 1e-4, 0.0], 0.0)                       # |e| <= e_tol
    assert not S([0.2, 0.1, 0.15], 0.0)                   # above 1/8 two steps back: keep going
    assert not S([0.1, 0.05, 0.06], 0.0)                  # 4 (0.1)^2 / 0.8^2 = 0.0625
    assert S([0.1, 0.05, 0.07], 0.0)
    assert not S([0.125, 0.05, 0.111], 0.0)               # 4/64 / (3/4)^2 = 0.1111...
    assert S([0.125, 0.05, 0.1112], 0.0)
    assert not S([0.1251, 0.05, 0.12], 0.0)               # just above 1/8
    assert S([5e-4, 1e-4, 5e-4], 0.0)                     # no decrease over two steps
    assert not S([5e-9, 1e-12, 9e-17], 0.0)               # squared: 9e-17 <= 4 (5e-9)^2 / (1 - 1e-8)^2
    assert S([5e-9, 1e-12, 2e-16], 0.0)                   # more: the noise floor
    assert S([-7.6e-9, 7.6e-10, -2.5e-10], 0.0)           # signs do not matter
