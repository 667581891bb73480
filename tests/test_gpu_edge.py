"""Edge cases through the C ABI against the oracle: empty matrices, a
threshold that skips every pair, a truncation budget above the whole norm,
a single ragged block (n < b), a diagonal F (the exact step function) and
the degenerate occupations n_occ = 0 and n_occ = n."""
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


@pytest.mark.parametrize("b", [32, 64])
def test_empty_matrix(b):
    n = 3 * b - 5
    E = oracle.BSM(n, b, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, b, b)))
    G = P.BlockSparse.from_host(E)
    P.build_norms(G)
    tl = synth.tau_log(16)
    for kind in ("tree", "flat", "sum"):
        bound, idx, tau = P.sweep_tau(G, G, tl, 1e-6, b_transposed=True, bound=kind)
        assert np.all(bound.cpu().numpy() == 0.0)
        assert int(idx.item()) == 0 and float(tau.item()) == tl[0]
    C, kept = P.multiply(G, G, 0.0, symmetric=True, b_transposed=True)
    assert int(kept[0].item()) == 0 and int(kept[1].item()) == 0
    assert to_oracle(C).nblk == 0
    out = P.truncate(G, 1e-3, sync=True)
    assert float(out[0].item()) == 0.0 and to_oracle(G).nblk == 0


def test_threshold_above_every_product():
    X = sym_x(700, 32, 5)
    G = P.BlockSparse.from_host(X)
    P.build_norms(G)
    nu = oracle.norms(X)[1]
    big = 2.0 * float(nu.max()) ** 2
    C, kept = P.multiply(G, G, big, symmetric=True, b_transposed=True)
    Co, K = oracle.spamm(X, X, big, sym=True)
    assert int(kept[0].item()) == 0 == K.npairs
    assert to_oracle(C).nblk == Co.nblk == 0
    # and the sweep bound at that threshold is the whole recursive bound of skipping everything
    bound, _, _ = P.sweep_tau(G, G, np.array([big]), 1e-30, b_transposed=True)
    assert bound.cpu().numpy()[0] == oracle.cse_tree(X, X, np.array([big]))[0] > 0.0


def test_truncation_budget_above_the_norm():
    X = sym_x(700, 32, 6)
    G = P.BlockSparse.from_host(X)
    P.build_norms(G)
    delta = 2.0 * np.linalg.norm(X.vals) + 1.0
    P.truncate(G, delta, sync=True)
    Xt, _ = oracle.truncate(X, delta)
    got = to_oracle(G)
    assert np.array_equal(got.keys(), Xt.sorted().keys())
    assert Xt.nblk == 0


def test_single_ragged_block():
    """n = 20 < b = 32: one block, mostly padding."""
    rng = np.random.default_rng(2)
    n, b = 20, 32
    A = rng.standard_normal((n, n))
    Fd = (A + A.T) / 2
    F = oracle.from_dense(Fd, b)
    w, U = np.linalg.eigh(Fd)
    n_occ = 9
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=synth.tau_log(32), homo=w[n_occ - 1], lumo=w[n_occ])
    Do, logs_o, _ = oracle.sp2(F, p)
    G = P.BlockSparse.from_host(F)
    res = P.purify(G, n_occ, 1e-6, synth.tau_log(32), homo=w[n_occ - 1], lumo=w[n_occ])
    assert [lg["branch"] for lg in res.logs] == [lo.branch for lo in logs_o]
    Dg = to_oracle(res.D).to_dense()
    assert np.abs(Dg - Do.to_dense()).max() < 1e-12
    assert np.linalg.norm(Dg - U[:, :n_occ] @ U[:, :n_occ].T) < 1e-6


def test_diagonal_f_exact_step_function():
    n, b = 96, 32
    rng = np.random.default_rng(0)
    f = rng.uniform(-2.0, 2.0, n)
    f[np.abs(f) < 0.3] += 0.6
    n_occ = int(np.sum(f < 0.0))
    F = oracle.from_dense(np.diag(f), b)
    fs = np.sort(f)
    G = P.BlockSparse.from_host(F)
    res = P.purify(G, n_occ, 1e-6, synth.tau_paper(), homo=fs[n_occ - 1], lumo=fs[n_occ])
    Dg = to_oracle(res.D).to_dense()
    assert np.array_equal(Dg, np.diag((f < 0.0).astype(np.float64)))
    assert np.trace(Dg) == n_occ


@pytest.mark.parametrize("occ", ["none", "all"])
def test_degenerate_occupation(occ):
    Fm = synth.chain1d(256, 3, 32)
    F = oracle.BSM.of(Fm)
    n = F.n
    n_occ = 0 if occ == "none" else n
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=synth.tau_paper(), delta_const=1e-9)
    Do, logs_o, _ = oracle.sp2(F, p)
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, n_occ, 1e-6, synth.tau_paper(), delta_const=1e-9)
    assert [lg["branch"] for lg in res.logs] == [lo.branch for lo in logs_o]
    Dg = to_oracle(res.D).to_dense()
    assert np.abs(Dg - Do.to_dense()).max() < 1e-12
    want = np.zeros((n, n)) if occ == "none" else np.eye(n)
    assert np.linalg.norm(Dg - want) < 1e-6


def test_tau_fallback_warning():
    """No candidate below the budget: the synchronising sweep and the
    purification return the SPAMM_WTAUFALLBACK warning with tau = 0 (the
    exact product), and the purification's steps equal the oracle's."""
    X = sym_x(1024, 32, 1)
    G = P.BlockSparse.from_host(X)
    P.build_norms(G)
    tl = synth.tau_log(8, -4.0)                       # 1 ... 1e-4
    bound, idx, tau, rc = P.sweep_tau(G, G, tl, 1e-30, b_transposed=True, sync=True, with_status=True)
    assert rc == P.SPAMM_WTAUFALLBACK and int(idx.item()) == len(tl) and float(tau.item()) == 0.0
    bound, idx, tau, rc = P.sweep_tau(G, G, tl, 1e30, b_transposed=True, sync=True, with_status=True)
    assert rc == P.SPAMM_OK and int(idx.item()) == 0
    Fm = synth.chain1d(512, 1, 32)
    F = oracle.BSM.of(Fm)
    p = oracle.SP2Params(n_occ=256, eps=1e-6, taus=tl, delta_const=1e-14)
    Do, logs_o, _ = oracle.sp2(F, p)
    assert any(l.branch >= 0 and l.idx == len(tl) for l in logs_o)
    res = P.purify(P.BlockSparse.from_host(Fm), 256, 1e-6, tl, delta_const=1e-14)
    assert res.status == P.SPAMM_WTAUFALLBACK
    assert [(l["branch"], l["idx"], l["npairs"]) for l in res.logs if l["branch"] >= 0] == \
        [(l.branch, l.idx, l.npairs) for l in logs_o if l.branch >= 0]
    assert np.abs(to_oracle(res.D).to_dense() - Do.to_dense()).max() < 1e-12
    # Algorithm 1 always runs the exact product: no warning
    res = P.purify(P.BlockSparse.from_host(Fm), 256, 1e-6, tl, delta_const=1e-14, variant="truncmul")
    assert res.status == P.SPAMM_OK


def test_x0_gerschgorin_radius_exactly_rounded():
    """A Gerschgorin row whose |f| sum 1 + 2^-53 + 2^-110 lies just above a
    rounding tie: double-double accumulation keeps 1 + 2^-53 and would round
    to 1, the exact sum rounds to 1 + 2^-52.  That row sets lambda_max, so
    X_0 is bit-identical to the oracle's only with the exactly rounded
    radius."""
    n, b = 64, 32
    Fd = np.diag(np.where(np.arange(n) % 2 == 0, 0.1, -0.1))
    Fd[5, 5] = 0.5
    for j, v in ((10, 1.0), (40, 2.0 ** -53), (50, 2.0 ** -110)):
        Fd[5, j] = Fd[j, 5] = v
    Fm = synth.BlockMatrix.from_dense(Fd, b)
    F = oracle.BSM.of(Fm)
    lmin, lmax = oracle.gerschgorin(F)
    assert lmax == 1.5 + 2.0 ** -52
    p = oracle.SP2Params(n_occ=n // 2, eps=1e-6, taus=synth.tau_log(16), delta_const=1e-300)
    X0o, _, _, _ = oracle.sp2_start(F, p)
    res = P.purify(P.BlockSparse.from_host(Fm), n // 2, 1e-6, synth.tau_log(16), delta_const=1e-300,
                   keep_tape=True, n_max=4)
    X0g = to_oracle(res.tape(0))
    assert np.array_equal(X0g.keys(), X0o.keys())
    assert np.array_equal(X0g.vals.view(np.uint64), X0o.sorted().vals.view(np.uint64))
