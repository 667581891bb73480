"""GPU parity of the reverse mode (frozen decisions, not in the paper)
through the C ABI:

* one step, teacher-forced on the GPU's own tape: Xbar against the oracle's
  adjoint_step within 1e-12 (relative Frobenius), pair and output counts
  exact, both branches, leaf 32 and 64, ragged n;
* the whole chain (purify_sp2_adjoint) against the oracle's sp2_adjoint run
  on the same tape and decisions;
* the autograd path returns exactly what the direct call returns;
* checkpoints every k iterates (segments recomputed in the backward pass)
  give exactly the full-tape gradient."""
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


def slot_values(M, val: torch.Tensor) -> np.ndarray:
    """Values of M's live blocks from a tensor in M's slot layout, in the
    sorted block order of to_oracle(M)."""
    _, _, _, _, _, o = M.live()
    b = M.b
    return val.detach().cpu().numpy().reshape(-1, b, b)[o]


def sym_random_on(M, rng):
    """Random symmetric values on the pattern of M: (tensor in M's slot
    layout, the same values as an oracle BSM)."""
    brow, bcol, _, _, _, o = M.live()
    b, n = M.b, M.n
    nn = M.nb * b
    R = rng.standard_normal((nn, nn))
    R = R + R.T
    R[n:, :] = 0.0
    R[:, n:] = 0.0
    vals = np.zeros((brow.shape[0], b, b))
    for t in range(brow.shape[0]):
        r, c = int(brow[t]), int(bcol[t])
        vals[t] = R[r * b:(r + 1) * b, c * b:(c + 1) * b].T
    g = np.zeros((M.cap, b, b))
    g[o] = vals
    gt = torch.from_numpy(g.reshape(-1)).to("cuda")
    return gt, oracle.BSM(n, b, brow, bcol, vals)


def forward(case):
    if case == "chain":
        Fm = synth.chain1d(1024, 1, 32)
        n_occ, taus = 512, synth.tau_paper()
    else:
        Fm = synth.sys3d(1500, 3, 64)
        n_occ, taus = 750, synth.tau_log(32)
    F = oracle.BSM.of(Fm)
    w = np.linalg.eigvalsh(F.to_dense())
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, n_occ, 1e-6, taus, homo=w[n_occ - 1], lumo=w[n_occ], keep_tape=True)
    return F, G, res


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("case", ["chain", "sys3d"])
def test_adjoint_step_teacher_forced(case):
    rng = np.random.default_rng(7)
    F, G, res = forward(case)
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    picks = sorted({0, len(steps) // 3, len(steps) // 2, len(steps) - 1})
    picks += [t for t in range(len(steps)) if steps[t]["branch"] == 1][:1]
    picks += [t for t in range(len(steps)) if steps[t]["branch"] == 0][:1]
    seen = set()
    for t0 in sorted(set(picks)):
        lg = steps[t0]
        X = res.tape(t0)
        S1 = res.tape(t0 + 1)
        gval, Go = sym_random_on(S1, rng)
        xbar, counts = P.adjoint_step(X, P.with_values(S1, gval), lg["tau"], lg["branch"])
        Xo = to_oracle(X)
        want = oracle.adjoint_step(Xo, Go, lg["tau"], lg["branch"])
        got = slot_values(X, xbar)
        assert rel(got, want.vals) <= 1e-12, (t0, lg["branch"])
        # counts: outputs are the live blocks with r <= c; pairs are the kept
        # triples with G_ac present, plus those with a == b once more
        c = counts.cpu().numpy()
        assert int(c[0]) == int(np.sum(Xo.brow <= Xo.bcol))
        nu = oracle.norms(Xo)[1]
        K = oracle.kept(Xo, Xo, lg["tau"], False, nu, nu)
        gm = Go.block_map()
        ng = nd = 0
        for o in range(K.oi.shape[0]):
            a, cc = int(K.oi[o]), int(K.oj[o])
            if gm[a * Xo.nb + cc] < 0:
                continue
            ks = K.klist[K.kptr[o]:K.kptr[o + 1]]
            ng += ks.shape[0]
            nd += int(np.sum(ks == a))
        assert int(c[1]) == ng + nd
        seen.add(lg["branch"])
    assert seen == {0, 1}


@pytest.mark.parametrize("case", ["chain", "sys3d"])
def test_purify_adjoint_against_oracle_chain(case):
    rng = np.random.default_rng(9)
    F, G, res = forward(case)
    ntape = res.nlog
    tape = [to_oracle(res.tape(t)) for t in range(ntape)]
    D = res.tape(ntape - 1)
    dval, Do = sym_random_on(D, rng)
    fbar = P.purify_adjoint(res, G, dval)

    class L:
        def __init__(self, lg):
            self.tau, self.branch = lg["tau"], lg["branch"]
    logs = [L(lg) for lg in res.logs]
    lmin, lmax = oracle.gerschgorin(F)
    want = oracle.sp2_adjoint(F, tape, logs, lmin, lmax, Do)
    got = slot_values(G, fbar)
    assert rel(got, want.vals) <= 1e-10
    assert np.linalg.norm(got) > 0.0


def test_autograd_matches_direct_call():
    rng = np.random.default_rng(4)
    Fm = synth.chain1d(512, 2, 32)
    F = oracle.BSM.of(Fm)
    w = np.linalg.eigvalsh(F.to_dense())
    G = P.BlockSparse.from_host(Fm)
    fval = G.val.clone().requires_grad_(True)
    dval, res = P.purify_autograd(G, fval, 256, 1e-6, synth.tau_paper(), homo=w[255], lumo=w[256])
    wt, _ = sym_random_on(res.D, rng)
    loss = (dval * wt).sum()
    loss.backward()
    direct = P.purify_adjoint(res, P.with_values(G, fval.detach()), wt)
    assert torch.equal(fval.grad, direct)
    assert float(fval.grad.abs().sum()) > 0.0


@pytest.mark.parametrize("every", [3, 4])
def test_checkpointed_adjoint_equals_full_tape(every):
    """Checkpoints every k iterates, segments recomputed in the backward pass
    with the recorded decisions by the forward's own kernels: the iterates
    are bit-identical, so the gradient equals the full-tape one exactly."""
    rng = np.random.default_rng(12)
    Fm = synth.sys3d(1500, 3, 64)
    F = oracle.BSM.of(Fm)
    w = np.linalg.eigvalsh(F.to_dense())
    G = P.BlockSparse.from_host(Fm)
    kw = dict(homo=w[749], lumo=w[750])
    full = P.purify(G, 750, 1e-6, synth.tau_log(32), keep_tape=True, **kw)
    ck = P.purify(G, 750, 1e-6, synth.tau_log(32), keep_tape=every, **kw)
    assert full.nlog - 1 > 2 * every             # several segments
    for a, b in zip(full.logs, ck.logs):
        assert a["npairs"] == b["npairs"] and a["tau"] == b["tau"] and a["branch"] == b["branch"]
    dval, _ = sym_random_on(full.D, rng)
    g_full = P.purify_adjoint(full, G, dval)
    g_ck = P.purify_adjoint(ck, G, dval)
    assert torch.equal(g_full, g_ck)
    assert float(g_ck.abs().sum()) > 0.0


def test_zero_tolerance_gradient_equals_dense_references():
    """With zero tolerances (tau = 0, nothing truncated) the GPU's dL/dF
    equals the dense FP64 chain rule of the SP2 polynomials with the run's
    branches and Gerschgorin bounds, and (SP2 having converged) the
    derivative of the exact spectral projector onto the n_occ lowest
    eigenvectors: sum over occupied a, virtual v of the (a, v) entry of
    U^T W U divided by e_a - e_v, on both (a, v) and (v, a)."""
    rng = np.random.default_rng(31)
    Fm = synth.chain1d(512, 2, 32)
    F = oracle.BSM.of(Fm)
    n, n_occ = F.n, 256
    G = P.BlockSparse.from_host(Fm)
    res = P.purify(G, n_occ, 1e-6, synth.tau_paper(), delta_const=0.0, n_max=40, keep_tape=True)
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    assert all(lg["tau"] == 0.0 for lg in steps) and len(steps) >= 10
    dval, Do = sym_random_on(res.D, rng)
    Wm = Do.to_dense()
    fbar = P.purify_adjoint(res, G, dval)
    got = np.zeros((n, n))
    vals = slot_values(G, fbar)
    brow, bcol, _, _, _, _ = G.live()
    mask = np.zeros((n, n), dtype=bool)
    b = F.b
    for t in range(brow.shape[0]):
        r, c = int(brow[t]), int(bcol[t])
        got[r * b:(r + 1) * b, c * b:(c + 1) * b] = vals[t].T
        mask[r * b:(r + 1) * b, c * b:(c + 1) * b] = True
    # dense chain rule with the run's own branches and bounds
    lmin, lmax = oracle.gerschgorin(F)
    Xs = [(lmax * np.eye(n) - F.to_dense()) / (lmax - lmin)]
    for lg in steps:
        X = Xs[-1]
        Xs.append(X @ X if lg["branch"] == 0 else 2 * X - X @ X)
    Gb = Wm.copy()
    for t in range(len(steps), 0, -1):
        X = Xs[t - 1]
        GX = Gb @ X + X @ Gb
        Gb = GX if steps[t - 1]["branch"] == 0 else 2 * Gb - GX
    want = -Gb / (lmax - lmin)
    assert np.linalg.norm((got - want)[mask]) <= 1e-10 * np.linalg.norm(want[mask])
    # the exact projector's derivative
    e, U = np.linalg.eigh(F.to_dense())
    Wt = U.T @ Wm @ U
    occ = np.arange(n) < n_occ
    Gam = np.zeros((n, n))
    de = e[:, None] - e[None, :]
    cross = occ[:, None] != occ[None, :]
    Gam[cross] = (occ[:, None].astype(float) - occ[None, :].astype(float))[cross] / de[cross]
    Fex = U @ (Gam * Wt) @ U.T
    assert np.linalg.norm((got - Fex)[mask]) <= 1e-8 * np.linalg.norm(Fex[mask])
