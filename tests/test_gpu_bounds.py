"""Leaf-level error bounds (B_flat: eq. (6) applied to the leaf blocks of
each output; B_sum: the plain sum of the skipped products) on the GPU
through the C ABI, against the oracle's triple loop.

Both sides form every product p = RN(nu_A nu_B) and every per-output sum
over k in ascending order the same way, and round the sum over the outputs
once from its exact value, so the bound vectors, the selections and every
purification step are compared bit for bit.  Sums that sit on a rounding
boundary (exact ties) take the GPU's exact fallback path."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2005_10680_amd as P  # noqa: E402

def to_oracle(M):
    brow, bcol, vals, _, _, _ = M.live()
    return oracle.BSM(M.n, M.b, brow, bcol, vals)


def sym_x(n, b, seed):
    F = oracle.BSM.of(synth.sys3d(n, seed, b))
    lmin, lmax = oracle.gerschgorin(F)
    return oracle.x0(F, lmin, lmax)


def same_bits(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), \
        np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300))


def budgets_for(bound):
    """Budgets at every distinct bound value (the strict < of the selection)
    and between consecutive ones, plus one above and one below them all."""
    vals = sorted(set(float(v) for v in bound if v > 0))
    out = [2.0 * vals[-1] if vals else 1.0, 1e-300]
    for t in range(len(vals)):
        out.append(vals[t])
        if t + 1 < len(vals):
            out.append(0.5 * (vals[t] + vals[t + 1]))
    return out


@pytest.mark.parametrize("kind", ["flat", "sum"])
@pytest.mark.parametrize("n,b,seed,taus", [
    (1024, 32, 1, "paper"),     # 350 candidates
    (1500, 32, 2, "log"),       # ragged tail
    (2048, 64, 3, "log"),
    (300, 128, 4, "log"),       # nb = 3
])
def test_leaf_bounds_symmetric(kind, n, b, seed, taus):
    X = sym_x(n, b, seed)
    tl = synth.tau_paper() if taus == "paper" else synth.tau_log(32)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    flat, ssum = oracle.cse_flat_sum(X, X, tl)
    want = flat if kind == "flat" else ssum
    bound, idx, tau = P.sweep_tau(M, M, tl, 1e-6, b_transposed=True, bound=kind)
    same_bits(bound.cpu().numpy(), want)
    tree = oracle.cse_tree(X, X, tl)
    assert np.all(flat <= tree * (1 + 1e-12)) and np.all(tree <= ssum * (1 + 1e-12))
    for budget in budgets_for(want):
        bound, idx, tau = P.sweep_tau(M, M, tl, budget, b_transposed=True, bound=kind)
        oi, ot = oracle.select(want, tl, budget)
        assert int(idx.item()) == oi and float(tau.item()) == ot


@pytest.mark.parametrize("kind", ["flat", "sum"])
def test_leaf_bounds_nonsymmetric_normal_layout(kind):
    rng = np.random.default_rng(7)
    n, b = 1000, 32
    A = sym_x(n, b, 5)
    Bh = oracle.BSM(A.n, b, A.brow, A.bcol, A.vals * rng.uniform(0.5, 2.0, size=(A.nblk, 1, 1)))
    Bh = Bh.subset(rng.random(Bh.nblk) < 0.7)
    tl = synth.tau_log(32)
    GA, GB = P.BlockSparse.from_host(A), P.BlockSparse.from_host(Bh)
    P.build_norms(GA)
    P.build_norms(GB)
    bound, _, _ = P.sweep_tau(GA, GB, tl, 1e-6, bound=kind)
    flat, ssum = oracle.cse_flat_sum(A, Bh, tl)
    same_bits(bound.cpu().numpy(), flat if kind == "flat" else ssum)


def test_leaf_bounds_deterministic_and_degenerate():
    X = sym_x(1500, 32, 2)
    tl = synth.tau_log(32)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    a = P.sweep_tau(M, M, tl, 1e-6, b_transposed=True, bound="flat")[0].cpu().numpy()
    b = P.sweep_tau(M, M, tl, 1e-6, b_transposed=True, bound="flat")[0].cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    # a threshold below every product skips nothing: both bounds are 0
    tiny = np.array([1e-300, 1e-310])
    for kind in ("flat", "sum"):
        bd, idx, tau = P.sweep_tau(M, M, tiny, 1e-20, b_transposed=True, bound=kind)
        assert np.all(bd.cpu().numpy() == 0.0) and int(idx.item()) == 0
    # a threshold above every product skips everything: B_sum is the sum of all products
    nu = oracle.norms(X)[1]
    big = np.array([2.0 * float(nu.max()) ** 2 + 1.0])
    bd = P.sweep_tau(M, M, big, 1e-6, b_transposed=True, bound="sum")[0].cpu().numpy()
    _, ssum = oracle.cse_flat_sum(X, X, big)
    same_bits(bd, ssum)


def test_leaf_bounds_rejected_arguments():
    X = sym_x(500, 32, 3)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    tl = torch.as_tensor(synth.tau_log(8), dtype=torch.float64, device="cuda")
    N = int(tl.shape[0])
    bound = torch.empty(N, dtype=torch.float64, device="cuda")
    idx = torch.empty(1, dtype=torch.int32, device="cuda")
    tau = torch.empty(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(P.lib().spamm_sweep_workspace_bytes(M.nb, N), dtype=torch.uint8, device="cuda")
    t0 = torch.zeros(1, dtype=torch.float64, device="cuda")

    def call(mode, flags):
        return P.lib().spamm_sweep_tau(ctypes.byref(M.struct()), ctypes.byref(M.struct()),
                                       ctypes.c_void_p(tl.data_ptr()), N, None, 1e-6, mode,
                                       ctypes.c_void_p(t0.data_ptr()), 0.5, flags,
                                       ctypes.c_void_p(bound.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                       ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                       ws.numel(), P._stream())
    both = P.B_TRANSPOSED | P.BOUND_FLAT | P.BOUND_SUM
    assert call(0, both) == P.SPAMM_EINVAL
    assert call(2, P.B_TRANSPOSED | P.BOUND_FLAT) == P.SPAMM_EINVAL
    assert call(0, P.B_TRANSPOSED | P.BOUND_SUM | P.SYNC) == P.SPAMM_OK
    assert call(1, P.B_TRANSPOSED | P.BOUND_FLAT | P.SYNC) == P.SPAMM_OK


@pytest.mark.parametrize("kind", ["flat", "sum"])
def test_leaf_bounds_tier_mode(kind):
    """Tier mode (skip p < tau0, c p from tau0 up to sigma_m) against the
    oracle's, for the FP32 and split-BF16 constants and several tau0."""
    X = sym_x(1500, 32, 2)
    tl = synth.tau_log(32)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    for prec in (1, 2):
        c = oracle.tier_constant(prec, 32)
        for t0 in (tl[10], tl[14], tl[20]):
            bound, idx, tau = P.sweep_tau(M, M, tl, 1e-7, b_transposed=True, mode=1, tau0=t0, c_low=c,
                                          bound=kind)
            f, sm = oracle.cse_flat_sum(X, X, tl, mode=1, tau0=t0, c_low=c)
            want = f if kind == "flat" else sm
            same_bits(bound.cpu().numpy(), want)
            for budget in budgets_for(want)[:12]:
                _, idx, tau = P.sweep_tau(M, M, tl, budget, b_transposed=True, mode=1, tau0=t0, c_low=c,
                                          bound=kind)
                oi, ot = oracle.select(want, tl, budget)
                assert int(idx.item()) == oi and float(tau.item()) == ot


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_tiers_with_leaf_bound_teacher_forced(precision):
    """Precision tiers selecting with B_flat, every step on the GPU's own
    iterate: tau, sigma and the kept / low-tier pair counts equal the
    oracle's; the run converges."""
    n, b = 2048, 64
    Fm = synth.sys3d(n, 12, b)
    F = oracle.BSM.of(Fm)
    w, Uv = np.linalg.eigh(F.to_dense())
    n_occ = n // 2
    taus = synth.tau_log(32)
    prec = P.PRECISIONS[precision]
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, homo=w[n_occ - 1], lumo=w[n_occ], precision=prec,
                         bound="flat")
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, n_occ, 1e-6, taus, homo=w[n_occ - 1], lumo=w[n_occ], keep_tape=True, precision=precision,
                   bound="flat")
    c = oracle.tier_constant(prec, b)
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    nlow = 0
    for t, lg in enumerate(steps):
        X = to_oracle(res.tape(t))
        nu = oracle.norms(X)[1]
        budget = lg["delta"] / 2.0
        f0, _ = oracle.cse_flat_sum(X, X, taus, nu, nu)
        idx, tau = oracle.select(f0, taus, p.tier_split * budget)
        assert lg["idx"] == idx and lg["tau"] == tau
        f1, _ = oracle.cse_flat_sum(X, X, taus, nu, nu, mode=1, tau0=tau, c_low=c)
        sidx, sigma = oracle.select(f1, taus, budget)
        assert lg["sidx"] == sidx and lg["sigma"] == sigma
        K = oracle.kept(X, X, tau, True, nu, nu)
        assert lg["npairs"] == K.npairs
        low = oracle.low_tier_pairs(X, tau, sigma, nu, prec)
        assert lg["npairs_low"] == low
        nlow += low
    assert nlow > 0
    Dref = Uv[:, :n_occ] @ Uv[:, :n_occ].T
    assert np.linalg.norm(to_oracle(res.D).to_dense() - Dref) < 1e-6


@pytest.mark.parametrize("kind", ["flat", "sum"])
def test_purify_leaf_bound_teacher_forced(kind):
    """Every step of the GPU run against the oracle's step with the same
    bound on the GPU's own previous iterate: branch, selection and kept-pair
    counts exact, iterates within 1e-12; the result converges."""
    n, b = 2048, 64
    Fm = synth.sys3d(n, 12, b)
    F = oracle.BSM.of(Fm)
    w, Uv = np.linalg.eigh(F.to_dense())
    n_occ = n // 2
    taus = synth.tau_log(32)
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, homo=w[n_occ - 1], lumo=w[n_occ], bound=kind)
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, n_occ, 1e-6, taus, homo=w[n_occ - 1], lumo=w[n_occ], keep_tape=True, bound=kind)
    _, _, st, _ = oracle.sp2_start(F, p)
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    assert len(steps) >= 8
    xh, xl, e_hist = st.xh, st.xl, []
    for t, lg in enumerate(steps):
        Xprev = to_oracle(res.tape(t))
        Xn, _, log, ost2 = oracle.sp2_step(Xprev, oracle.SP2State(t + 1, xh, xl, list(e_hist)), p)
        assert Xn is not None and lg["branch"] == log.branch
        assert lg["idx"] == log.idx and lg["tau"] == log.tau
        assert lg["npairs"] == log.npairs and lg["nout"] == log.nout
        Xg = to_oracle(res.tape(t + 1))
        assert np.array_equal(Xg.keys(), Xn.keys())
        d = np.linalg.norm(Xg.vals - Xn.vals)
        assert d <= 1e-12 * np.linalg.norm(Xn.vals)
        xh, xl, e_hist = ost2.xh, ost2.xl, ost2.e_hist
    Dref = Uv[:, :n_occ] @ Uv[:, :n_occ].T
    assert np.linalg.norm(to_oracle(res.D).to_dense() - Dref) < 1e-6


def test_leaf_bound_graph_and_batch_match_host_loop():
    """The graph-captured loop and the batched driver take the same
    decisions with a leaf-level bound as the host loop does, also with a
    precision tier (sigma selected with the same bound)."""
    cases = [(synth.sys3d(1500, 21, 64), "flat", "fp64"), (synth.chain1d(1024, 4, 32), "sum", "fp64"),
             (synth.sys3d(1200, 22, 32), "tree", "fp64"), (synth.sys3d(1400, 23, 64), "flat", "bf16x3"),
             (synth.sys3d(1100, 24, 32), "sum", "fp32")]
    Fs, data = [], []
    for Fm, kind, prec in cases:
        w = np.linalg.eigvalsh(oracle.BSM.of(Fm).to_dense())
        n = Fm.n
        Fs.append(P.BlockSparse.from_host(Fm))
        data.append((n // 2, w[n // 2 - 1], w[n // 2], kind, prec))
    taus = synth.tau_log(32)
    singles = [P.purify(F, d[0], 1e-6, taus, homo=d[1], lumo=d[2], bound=d[3], precision=d[4])
               for F, d in zip(Fs, data)]
    for F, d, s in zip(Fs, data, singles):
        g = P.purify(F, d[0], 1e-6, taus, homo=d[1], lumo=d[2], bound=d[3], precision=d[4], graph_steps=4)
        for f in ("tau", "sigma", "npairs", "npairs_low"):
            assert [lg[f] for lg in g.logs] == [lg[f] for lg in s.logs], f
        assert np.array_equal(g.D.live()[2], s.D.live()[2])
    assert sum(lg["npairs_low"] for lg in singles[3].logs) > 0
    res = P.purify_batched(Fs, [d[0] for d in data], 1e-6, taus, [d[1] for d in data], [d[2] for d in data],
                           bound=[d[3] for d in data], precision=[d[4] for d in data], graph_steps=4)
    assert res.rc == P.SPAMM_OK
    for q, s in enumerate(singles):
        for f in ("tau", "sigma", "npairs", "npairs_low"):
            assert [lg[f] for lg in res.logs[q]] == [lg[f] for lg in s.logs], (q, f)
        assert np.array_equal(res.D[q].live()[2], s.D.live()[2])
    # the leaf-level bounds admit larger thresholds than the recursive one
    t_flat = P.purify(Fs[0], data[0][0], 1e-6, taus, homo=data[0][1], lumo=data[0][2], bound="flat")
    t_tree = P.purify(Fs[0], data[0][0], 1e-6, taus, homo=data[0][1], lumo=data[0][2], bound="tree")
    assert t_flat.logs[0]["tau"] >= t_tree.logs[0]["tau"]


def _diag_single(nb, b, values):
    vals = np.zeros((nb, b, b))
    vals[:, 0, 0] = values
    idx = np.arange(nb, dtype=np.int32)
    return oracle.BSM(nb * b, b, idx, idx.copy(), vals)


@pytest.mark.parametrize("case", ["sum_tie", "flat_tie", "sum_above", "flat_above"])
def test_leaf_bounds_on_rounding_boundaries(case):
    """Sums over outputs that are exact ties (1 + 2^-53: the double-double
    value cannot certify its rounding, so the exact fallback decides: to
    even) or just above one (1 + 2^-52 from three terms): equal to the
    oracle bit for bit."""
    b = 32
    va, vb, kind = {
        "sum_tie": ([1.0, 2.0 ** -26], [1.0, 2.0 ** -27], "sum"),
        "flat_tie": ([1.0, 2.0 ** -13, 2.0 ** -13], [1.0, 2.0 ** -14, 2.0 ** -14], "flat"),
        "sum_above": ([1.0, 2.0 ** -26, 2.0 ** -26], [1.0, 2.0 ** -27, 2.0 ** -27], "sum"),
        "flat_above": ([1.0] + [2.0 ** -14] * 32, [1.0] + [2.0 ** -14] * 32, "flat"),
    }[case]
    A, B = _diag_single(len(va), b, va), _diag_single(len(vb), b, vb)
    GA, GB = P.BlockSparse.from_host(A), P.BlockSparse.from_host(B)
    P.build_norms(GA)
    P.build_norms(GB)
    tl = np.array([4.0, 0.5])
    flat, ssum = oracle.cse_flat_sum(A, B, tl)
    want = flat if kind == "flat" else ssum
    bound, _, _ = P.sweep_tau(GA, GB, tl, 1e-6, bound=kind)
    same_bits(bound.cpu().numpy(), want)
    if case.endswith("tie"):
        assert want[0] == 1.0
