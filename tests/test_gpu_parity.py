"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars: bit-exact norms, bounds, selected candidate, kept sets, output
patterns and truncation sets; leaf-product values within 1e-12 relative
Frobenius error (FP64)."""
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


def to_oracle(M: "P.BlockSparse") -> oracle.BSM:
    brow, bcol, vals, _, _, _ = M.live()
    return oracle.BSM(M.n, M.b, brow, bcol, vals)


def gpu_norms(M):
    brow, bcol, vals, nrm, sq, _ = M.live()
    return brow, bcol, nrm, sq


def rel_fro(a, b):
    d = np.linalg.norm(a - b)
    s = np.linalg.norm(b)
    return d / s if s > 0 else d


def sym_x(n, b, seed):
    """A symmetric matrix shaped like an SP2 iterate: X_0 of a 3D system."""
    F = oracle.BSM.of(synth.sys3d(n, seed, b))
    lmin, lmax = oracle.gerschgorin(F)
    return oracle.x0(F, lmin, lmax)


# ---------------------------------------------------------------------------
# K1 norms
# ---------------------------------------------------------------------------

def tie_block(rng, b, scale_exp):
    """A b x b block of integers times 2^scale_exp whose exact sum of squares
    has 55 significant bits ending in binary 10: a rounding tie.  The sum of
    squares is 2 mod 4 when the count of odd entries is.  The last entry is
    zero."""
    amp = {32: 2.0 ** 22, 64: 2.0 ** 21, 128: 2.0 ** 20}[b]
    while True:
        a = np.round(rng.standard_normal((b, b)) * amp)
        a[b - 1, b - 1] = 0.0
        odd = int(np.sum(np.abs(a) % 2 == 1))
        k = 0
        while odd % 4 != 2:
            i, j = divmod(k, b)
            k += 1
            if a[i, j] % 2 == 0:
                a[i, j] += 1
                odd += 1
        S = sum(int(x) ** 2 for x in a.ravel())
        if 2 ** 54 <= S < 2 ** 55:
            return a * 2.0 ** scale_exp


@pytest.mark.parametrize("b", [32, 64, 128])
def test_norms_bitwise(b):
    rng = np.random.default_rng(b)
    nblk = 40
    vals = rng.standard_normal((nblk, b, b)) * np.exp(rng.uniform(-40, 3, size=(nblk, 1, 1)))
    vals[1] = 0.0
    vals[2] = 0.0
    vals[2][0, 0] = 1.0
    vals[2][0, 1] = 2.0 ** -27       # 1 + 2^-53: a tie, rounds to 1
    vals[2][0, 2] = 2.0 ** -27
    vals[3] = vals[2]
    vals[3][0, 3] = 2.0 ** -600      # just above the tie: rounds up
    vals[4] = 0.0
    vals[4][5, 7] = 5e-324           # subnormals only
    vals[4][6, 7] = 1e-310
    vals[5] *= 1e-170                # squares below the normal range
    vals[6] = 1e-300
    vals[7] = 0.0
    vals[7][0, 0] = 1.0
    vals[7][0, 1] = 2.0 ** -27
    vals[7][0, 2] = 2.0 ** -27
    vals[7][0, 3] = 2.0 ** -200      # above the tie by 2^-400: no double-double holds the sum
    for q in range(8, 12):           # integer entries whose exact sum of squares is a tie
        vals[q] = tie_block(rng, b, -30 - 4 * q)
    vals[12] = vals[8]
    vals[12][b - 1, b - 1] = 2.0 ** -200   # the same tie plus 2^-400: rounds upward
    brow = np.arange(nblk, dtype=np.int32) % 7
    bcol = np.arange(nblk, dtype=np.int32) // 7
    M = P.BlockSparse.from_blocks(7 * b, b, brow, bcol, vals)
    P.build_norms(M)
    _, _, nrm, sq = gpu_norms(M)
    O = oracle.BSM(7 * b, b, brow, bcol, vals).sorted()
    osq, onu = oracle.norms(O)
    assert np.array_equal(sq.view(np.uint64), osq.view(np.uint64))
    assert np.array_equal(nrm.view(np.uint64), onu.view(np.uint64))


def test_norms_nan_block():
    b = 32
    vals = np.ones((2, b, b))
    vals[1, 3, 4] = np.nan
    M = P.BlockSparse.from_blocks(2 * b, b, np.array([0, 1], np.int32), np.array([0, 1], np.int32), vals)
    P.build_norms(M)
    _, _, nrm, sq = gpu_norms(M)
    assert sq[0] == b * b and math.isnan(sq[1]) and math.isnan(nrm[1])


# ---------------------------------------------------------------------------
# K2 sweep (Algorithm 3) and selection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 64, 65, 1024])
@pytest.mark.parametrize("mode", [0, 1])
def test_sweep_bitwise_candidate_counts(N, mode):
    """The shortest and the longest candidate list (1 and 1024), and both
    sides of the cube pass's switch from one thread per candidate (N <= 64)
    to eight per candidate in slices of 32 (N = 65: a ragged last slice);
    Algorithm 3 alone (mode 0) and with the precision tier's leaf values
    (mode 1: p below tau0, c_low p from tau0 up to the candidate): the
    whole bound vector bitwise and the selection."""
    X = sym_x(1500, 32, 2)                         # nb = 47
    tl = np.array([1e-6]) if N == 1 else synth.tau_log(N, -20.0)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    kw = dict(mode=1, tau0=1e-9, c_low=0.25) if mode else {}
    obound = oracle.cse_tree(X, X, tl, **kw)
    for budget in [obound[N // 3] * 1.0000001, 1e-12, 1e-30]:
        bound, idx, tau = P.sweep_tau(M, M, tl, budget, b_transposed=True, **kw)
        gb = bound.cpu().numpy()
        assert np.array_equal(gb.view(np.uint64), obound.view(np.uint64))
        oi, ot = oracle.select(obound, tl, budget)
        assert int(idx.item()) == oi and float(tau.item()) == ot


@pytest.mark.parametrize("n,b,seed,taus", [
    (1024, 32, 1, "paper"),     # chain-sized, 350 candidates
    (1500, 32, 2, "log"),       # nb = 47, ragged tail
    (2048, 64, 3, "log"),
    (300, 128, 4, "log"),       # nb = 3
])
def test_sweep_bitwise(n, b, seed, taus):
    X = sym_x(n, b, seed)
    tl = synth.tau_paper() if taus == "paper" else synth.tau_log(32)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    obound = oracle.cse_tree(X, X, tl)
    for budget in [obound[len(tl) // 3] * 1.0000001, 1e-9, 1e-30]:
        bound, idx, tau = P.sweep_tau(M, M, tl, budget, b_transposed=True)
        gb = bound.cpu().numpy()
        assert np.array_equal(gb.view(np.uint64), obound.view(np.uint64))
        oi, ot = oracle.select(obound, tl, budget)
        assert int(idx.item()) == oi and float(tau.item()) == ot


def test_sweep_nonsymmetric_normal_layout():
    rng = np.random.default_rng(7)
    n, b = 1000, 32
    A = sym_x(n, b, 5)
    Bh = oracle.BSM(A.n, b, A.brow, A.bcol, A.vals * rng.uniform(0.5, 2.0, size=(A.nblk, 1, 1)))
    keep = rng.random(Bh.nblk) < 0.7
    Bh = Bh.subset(keep)
    tl = synth.tau_log(32)
    GA, GB = P.BlockSparse.from_host(A), P.BlockSparse.from_host(Bh)
    P.build_norms(GA); P.build_norms(GB)
    bound, idx, tau = P.sweep_tau(GA, GB, tl, 1e-6)
    ob = oracle.cse_tree(A, Bh, tl)
    assert np.array_equal(bound.cpu().numpy().view(np.uint64), ob.view(np.uint64))


# ---------------------------------------------------------------------------
# K3 multiply
# ---------------------------------------------------------------------------

def oracle_kept_set(K):
    s = set()
    for m in range(K.oi.shape[0]):
        for q in range(K.kptr[m], K.kptr[m + 1]):
            s.add((int(K.oi[m]), int(K.klist[q]), int(K.oj[m])))
    return s


@pytest.mark.parametrize("n,b,seed,q", [(1024, 32, 1, 0.5), (2000, 64, 2, 0.3), (640, 128, 3, 0.5),
                                        (1500, 32, 4, 0.0)])
def test_multiply_symmetric_parity(n, b, seed, q):
    X = sym_x(n, b, seed)
    _, nu = oracle.norms(X)
    tau = float(np.quantile(nu, q)) ** 2 if q > 0 else 0.0
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    C, kept = P.multiply(M, M, tau, symmetric=True, b_transposed=True)
    Co, Ko = oracle.spamm(X, X, tau, sym=True)
    kg = kept.cpu().numpy()
    assert int(kg[0]) == Ko.npairs and int(kg[1]) == Ko.oi.shape[0]
    G = to_oracle(C)
    assert np.array_equal(G.keys(), Co.keys())           # output pattern, bit-exact
    assert rel_fro(G.vals, Co.vals) <= 1e-12
    D = G.to_dense()
    assert np.array_equal(D, D.T)                          # mirrored blocks exact


@pytest.mark.parametrize("b", [32, 64])
def test_multiply_general_parity(b):
    rng = np.random.default_rng(11)
    n = 20 * b - 5
    A = sym_x(n, b, 9)
    Bh = oracle.BSM(A.n, b, A.brow, A.bcol, rng.standard_normal(A.vals.shape) * A.vals)
    Bh = Bh.subset(rng.random(Bh.nblk) < 0.8)
    _, nuA = oracle.norms(A)
    _, nuB = oracle.norms(Bh)
    tau = float(np.median(nuA)) * float(np.median(nuB))
    GA, GB = P.BlockSparse.from_host(A), P.BlockSparse.from_host(Bh)
    P.build_norms(GA); P.build_norms(GB)
    C, kept = P.multiply(GA, GB, tau)
    Co, Ko = oracle.spamm(A, Bh, tau, sym=False)
    G = to_oracle(C)
    assert int(kept[0].item()) == Ko.npairs
    assert np.array_equal(G.keys(), Co.keys())
    assert rel_fro(G.vals, Co.vals) <= 1e-12


def test_multiply_deterministic_and_tau_zero_dense():
    X = sym_x(1024, 32, 3)
    M = P.BlockSparse.from_host(X)
    P.build_norms(M)
    C1, _ = P.multiply(M, M, 0.0, symmetric=True, b_transposed=True)
    C2, _ = P.multiply(M, M, 0.0, symmetric=True, b_transposed=True)
    g1, g2 = C1.to_host(), C2.to_host()
    assert np.array_equal(g1.vals.view(np.uint64), g2.vals.view(np.uint64))
    Xd = X.to_dense()
    ref = Xd @ Xd
    got = to_oracle(C1).to_dense()
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


# ---------------------------------------------------------------------------
# K4 truncation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,b,seed", [(1024, 32, 1), (2000, 64, 2)])
def test_truncate_bitwise(n, b, seed):
    X = sym_x(n, b, seed)
    C, _ = oracle.spamm(X, X, 0.0, sym=True)              # a product with fill-in
    sq, _ = oracle.norms(C)
    tot = math.sqrt(float(np.sum(sq)))
    for delta in [tot * 1e-10, tot * 1e-6, tot * 1e-3, 0.0]:
        M = P.BlockSparse.from_host(C)
        P.build_norms(M)
        out = P.truncate(M, delta)
        Ot, info = oracle.truncate(C, delta)
        G = to_oracle(M)
        assert np.array_equal(G.keys(), Ot.keys())
        assert int(out[0].item()) == info.removed_keys.shape[0]


# ---------------------------------------------------------------------------
# purification
# ---------------------------------------------------------------------------

def test_purify_chain_matches_oracle():
    Fm = synth.chain1d(1024, 1, 32)
    F = oracle.BSM.of(Fm)
    w, U = np.linalg.eigh(F.to_dense())
    Dref = U[:, :512] @ U[:, :512].T
    taus = synth.tau_paper()
    p = oracle.SP2Params(n_occ=512, eps=1e-6, taus=taus, homo=w[511], lumo=w[512])
    Do, logs_o, _ = oracle.sp2(F, p)
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, 512, 1e-6, taus, homo=w[511], lumo=w[512])
    logs_g = res.logs
    assert len(logs_g) == len(logs_o)
    for lg, lo in zip(logs_g, logs_o):
        assert lg["branch"] == lo.branch
        if lo.branch >= 0:
            assert lg["idx"] == lo.idx and lg["tau"] == lo.tau
            assert lg["npairs"] == lo.npairs
            assert lg["delta"] == lo.delta
    Dg = to_oracle(res.D)
    assert np.array_equal(Dg.keys(), Do.keys())
    assert np.abs(Dg.to_dense() - Do.to_dense()).max() < 1e-12
    assert np.linalg.norm(Dg.to_dense() - Dref) < 1e-6


def test_purify_teacher_forced_steps():
    n, b = 2048, 64
    Fm = synth.sys3d(n, 12, b)
    F = oracle.BSM.of(Fm)
    w = np.linalg.eigvalsh(F.to_dense())
    n_occ = n // 2
    taus = synth.tau_log(32)
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, homo=w[n_occ - 1], lumo=w[n_occ])
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, n_occ, 1e-6, taus, homo=w[n_occ - 1], lumo=w[n_occ], keep_tape=True, n_max=60)
    logs = res.logs
    # X~_0 against the oracle's start
    X0o, _, st, _ = oracle.sp2_start(F, p)
    X0g = to_oracle(res.tape(0))
    assert np.array_equal(X0g.keys(), X0o.keys())
    assert np.array_equal(X0g.vals.view(np.uint64), X0o.sorted().vals.view(np.uint64))   # bit for bit
    steps = [lg for lg in logs if lg["branch"] >= 0]
    assert len(steps) >= 8
    xh, xl = st.xh, st.xl
    e_hist = []
    for t, lg in enumerate(steps):
        Xprev = to_oracle(res.tape(t))
        ost = oracle.SP2State(t + 1, xh, xl, list(e_hist))
        Xn, Xh, log, ost2 = oracle.sp2_step(Xprev, ost, p)
        assert Xn is not None
        assert lg["branch"] == log.branch
        assert lg["idx"] == log.idx and lg["tau"] == log.tau
        assert lg["npairs"] == log.npairs and lg["nout"] == log.nout
        T = res.tape(t + 1)
        Xg = to_oracle(T)
        assert np.array_equal(Xg.keys(), Xn.keys())
        assert lg["nslot_kept"] == Xn.nblk and lg["nslot_hat"] == Xh.nblk      # block counts of X~_i, X^_i
        assert rel_fro(Xg.vals, Xn.vals) <= 1e-12
        # the iterate's norms (from the product epilogue) are the exactly
        # rounded norms of its own values
        _, _, _, nrm, sq, _ = T.live()
        osq, onu = oracle.norms(Xg)
        assert np.array_equal(sq.view(np.uint64), osq.view(np.uint64))
        assert np.array_equal(nrm.view(np.uint64), onu.view(np.uint64))
        xh, xl, e_hist = ost2.xh, ost2.xl, ost2.e_hist
