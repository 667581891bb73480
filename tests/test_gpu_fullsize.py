"""Parity at full size, in the configuration the benchmark times.

The oracle cannot run whole purifications at these sizes, so every check
here is teacher-forced on the GPU's own iterates (kept in the run's tape)
and uses only what the oracle computes quickly at any size:

* 3D system n = 16384, leaf 64, seed 2, FP64 (the benchmark workload): the
  run with a tape equals the run without one bit for bit; at sampled steps
  the norms, traces, branch, delta, the whole Algorithm 3 bound vector, the
  selected candidate and the kept-pair counts equal the oracle's; sampled
  blocks of the next iterate equal the oracle's products combined with the
  step polynomial within a rounding bound; blocks the truncation removed
  are below its budget; a mid-run iterate truncated by the library and by
  the oracle loses exactly the same blocks; the result has trace n_occ, is
  idempotent and commutes with F.  The accuracy half of the workload's
  metric: ||D~ - D||_F < eps for FP64, both tiers and B_flat, against the
  exact projector from a dense eigensolver (a library routine, run on the
  GPU: the dense matrix is 2 GB).
* 3D system n = 65536, leaf 64, seed 3, FP64 and both precision tiers:
  the first step, with the same checks; in the tiers the sampled
  blocks are within the per-block tier bound (c times the sum of the norm
  products of the pairs evaluated in the low tier) of the FP64 oracle.

Rounding bars: a block of a product is a sum of kept b x b products; the
GPU and the oracle add the same terms in different orders, so they differ
by at most about (k b) u sum_k ||A_ik|| ||B_kj|| (k kept pairs, u = 2^-53);
1e-12 times the sum of the pairs' norm products covers k b up to 9000."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2005_10680_amd as P  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
REL = 1e-12


def to_oracle(M):
    brow, bcol, vals, nrm, _, _ = M.live()
    return oracle.BSM(M.n, M.b, brow, bcol, vals), nrm


def check_step(X, nu_gpu, lg, xh, xl, p, Xnext, rng, nsample=24):
    """All checks of one step X~_{t} -> X~_{t+1} (the latter on the GPU)."""
    nu = oracle.norms(X)[1]
    assert np.array_equal(nu.view(np.uint64), nu_gpu.view(np.uint64))
    t1, t2, e = oracle.traces(X)
    assert abs(lg["t1"] - t1) <= 2.0 ** -52 * abs(t1) and abs(lg["t2"] - t2) <= 2.0 ** -52 * abs(t2)
    br = oracle.choose_branch(lg["t1"], lg["t2"], p.n_occ)
    assert lg["branch"] == br
    assert lg["branch"] == oracle.choose_branch(t1, t2, p.n_occ)
    delta = oracle.step_delta(p, oracle.map_gap(xh, br) - oracle.map_gap(xl, br))
    assert lg["delta"] == delta
    budget = delta / 2.0
    taus = np.asarray(p.taus, dtype=np.float64)
    bound = oracle.cse_tree(X, X, taus, nu, nu)
    skip_budget = p.tier_split * budget if p.precision else budget
    idx, tau = oracle.select(bound, taus, skip_budget)
    assert lg["idx"] == idx and lg["tau"] == tau
    K = oracle.kept(X, X, tau, True, nu, nu)
    assert lg["npairs"] == K.npairs and lg["nout"] == K.oi.shape[0]
    c_low, sigma = 0.0, 0.0
    if p.precision:
        c_low = oracle.tier_constant(p.precision, X.b)
        bound2 = oracle.cse_tree(X, X, taus, nu, nu, mode=1, tau0=tau, c_low=c_low)
        sidx, sigma = oracle.select(bound2, taus, budget)
        assert lg["sidx"] == sidx and lg["sigma"] == sigma
        nlow = oracle.low_tier_pairs(X, tau, sigma, nu, p.precision)
        assert lg["npairs_low"] == nlow
    # sampled output blocks: the longest k list, the first and last outputs,
    # random ones that the truncation kept and random ones it removed
    lens = K.kptr[1:] - K.kptr[:-1]
    kept_out = Xnext.block_map()[K.oi.astype(np.int64) * X.nb + K.oj] >= 0
    on, off = np.nonzero(kept_out)[0], np.nonzero(~kept_out)[0]
    sel = {int(np.argmax(lens)), 0, K.oi.shape[0] - 1}
    sel |= set(rng.choice(on, size=min(nsample, on.shape[0]), replace=False).tolist())
    sel |= set(rng.choice(off, size=min(nsample // 3, off.shape[0]), replace=False).tolist())
    sel = np.array(sorted(sel), dtype=np.int64)
    C = oracle.block_products(X, X, K, sel)
    xmap = X.block_map()
    oi, oj = K.oi[sel].astype(np.int64), K.oj[sel].astype(np.int64)
    present, got = Xnext.blocks_at(oi, oj)
    checked = 0
    for t, s in enumerate(sel):
        i, j = int(oi[t]), int(oj[t])
        ks = K.klist[K.kptr[s]:K.kptr[s + 1]].astype(np.int64)
        pk = nu[xmap[i * X.nb + ks]] * nu[xmap[ks * X.nb + j]]
        xs = xmap[i * X.nb + j]
        xij = X.vals[xs] if xs >= 0 else np.zeros((X.b, X.b))
        want = C[t] if br == 0 else 2.0 * xij - C[t]
        low = float(np.sum(pk[(pk >= tau) & (pk < sigma)])) if p.precision else 0.0
        tol = REL * (float(np.sum(pk)) + 2.0 * np.linalg.norm(xij)) + c_low * low
        if not present[t]:
            # removed by the truncation: its whole norm counts against delta/2
            assert np.linalg.norm(want) < budget + tol
            continue
        assert np.linalg.norm(got[t] - want) <= tol, (i, j, np.linalg.norm(got[t] - want), tol)
        checked += 1
    assert checked >= min(nsample, on.shape[0])
    return br


# ---------------------------------------------------------------------------
# n = 16384, FP64: the benchmark workload
# ---------------------------------------------------------------------------

def test_sys3d_16384_fp64_full_run():
    n, b, seed = 16384, 64, 2
    with open(os.path.join(HERE, "golden", "spectra.json")) as f:
        spec = json.load(f)[f"sys3d_n{n}_s{seed}_b{b}"]
    Fm = synth.sys3d(n, seed, b)
    F = oracle.BSM.of(Fm)
    G = P.BlockSparse.from_host(Fm)
    n_occ, taus = n // 2, synth.tau_log(32)
    kw = dict(homo=spec["homo"], lumo=spec["lumo"])
    plain = P.purify(G, n_occ, 1e-6, taus, **kw)                      # as timed
    peak = max(max(lg["nslot_hat"], lg["nslot_kept"]) for lg in plain.logs)
    res = P.purify(G, n_occ, 1e-6, taus, keep_tape=True, cap=int(peak * 1.05) + 64, **kw)
    assert len(res.logs) == len(plain.logs)
    for a, c in zip(plain.logs, res.logs):
        for k in ("branch", "idx", "tau", "delta", "t1", "t2", "npairs", "nout", "nslot_kept"):
            assert a[k] == c[k], k
    pa, pc = plain.D.live(), res.D.live()
    assert all(np.array_equal(x, y) for x, y in zip(pa[:3], pc[:3]))
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, **kw)
    X0o, _, st, _ = oracle.sp2_start(F, p)
    X0g, _ = to_oracle(res.tape(0))
    assert np.array_equal(X0g.keys(), X0o.keys())
    assert np.array_equal(X0g.vals.view(np.uint64), X0o.sorted().vals.view(np.uint64))   # bit for bit
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    assert len(steps) >= 30
    picks = set(range(0, len(steps), 5)) | {1, 2, len(steps) - 2, len(steps) - 1}
    rng = np.random.default_rng(16384)
    xh, xl = st.xh, st.xl
    for t, lg in enumerate(steps):
        if t in picks:
            X, nu_g = to_oracle(res.tape(t))
            check_step(X, nu_g, lg, xh, xl, p, res.tape(t + 1), rng)
        xh, xl = oracle.map_gap(xh, lg["branch"]), oracle.map_gap(xl, lg["branch"])
    # truncation at full size: a mid-run iterate truncated by the library and
    # by the oracle at several budgets removes exactly the same blocks
    mid = len(steps) // 2
    Xm, _ = to_oracle(res.tape(mid))
    tot = float(np.sqrt(np.sum(oracle.norms(Xm)[0])))
    for delta in (tot * 1e-9, tot * 1e-6, tot * 1e-3):
        M = P.BlockSparse.from_host(Xm)
        P.build_norms(M)
        out = P.truncate(M, delta)
        Ot, info = oracle.truncate(Xm, delta)
        Mo, _ = to_oracle(M)
        assert np.array_equal(Mo.keys(), Ot.sorted().keys())
        assert int(out[0].item()) == info.removed_keys.shape[0]
        del M
    del Xm
    # properties of the result at any size: trace, idempotency, commutation with F
    D = res.D
    Do, _ = to_oracle(D)
    assert abs(oracle.traces(Do)[0] - n_occ) < 1e-6
    D2, _ = P.multiply(D, D, 0.0, symmetric=True, b_transposed=True)
    a = Do.to_dense()
    d2, _ = to_oracle(D2)
    assert np.linalg.norm(d2.to_dense() - a) < 1e-6
    del d2
    FD, _ = P.multiply(G, D, 0.0, b_transposed=True)
    fd, _ = to_oracle(FD)
    fdd = fd.to_dense()
    assert np.linalg.norm(fdd - fdd.T) < 1e-5
    del res, plain, D2, FD
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def sys3d_16384_projector():
    """F (device block-sparse) and the exact projector onto its n/2 lowest
    eigenvectors, dense on the GPU."""
    n, b, seed = 16384, 64, 2
    with open(os.path.join(HERE, "golden", "spectra.json")) as f:
        spec = json.load(f)[f"sys3d_n{n}_s{seed}_b{b}"]
    Fm = synth.sys3d(n, seed, b)
    G = P.BlockSparse.from_host(Fm)
    Fd = torch.from_numpy(oracle.BSM.of(Fm).to_dense()).cuda()
    w, U = torch.linalg.eigh(Fd)
    del Fd
    # the dense eigenvalues bracket the same gap as the stored spectrum
    assert abs(float(w[n // 2 - 1]) - spec["homo"]) < 1e-9 and abs(float(w[n // 2]) - spec["lumo"]) < 1e-9
    Uo = U[:, : n // 2].contiguous()
    del U, w
    Dref = Uo @ Uo.T
    del Uo
    yield n, b, G, spec, Dref
    del G, Dref
    torch.cuda.empty_cache()


def dense_on_gpu(M, n):
    """Dense copy of a block-sparse result (n a multiple of the leaf)."""
    brow, bcol, vals, _, _, _ = M.live()
    b, nb = M.b, n // M.b
    D = torch.zeros((nb, nb, b, b), dtype=torch.float64, device="cuda")
    v = torch.from_numpy(np.ascontiguousarray(vals.transpose(0, 2, 1))).cuda()   # [k, row, col]
    D[torch.from_numpy(brow.astype(np.int64)).cuda(), torch.from_numpy(bcol.astype(np.int64)).cuda()] = v
    return D.permute(0, 2, 1, 3).reshape(n, n)


@pytest.mark.parametrize("precision,bound", [("fp64", "tree"), ("fp32", "tree"), ("bf16x3", "tree"),
                                             ("fp64", "flat"), ("bf16x3", "flat")])
def test_sys3d_16384_accuracy(sys3d_16384_projector, precision, bound):
    n, b, G, spec, Dref = sys3d_16384_projector
    res = P.purify(G, n // 2, 1e-6, synth.tau_log(32), homo=spec["homo"], lumo=spec["lumo"], precision=precision,
                   bound=bound)
    assert res.status == P.SPAMM_OK
    err = float(torch.linalg.norm(dense_on_gpu(res.D, n) - Dref).item())
    assert err < 1e-6, err
    if precision != "fp64":
        assert sum(lg["npairs_low"] for lg in res.logs) > 0
    del res
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# n = 65536: the mixed-precision workload (first step)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sys3d_65536():
    n, b, seed = 65536, 64, 3
    Fm = synth.sys3d(n, seed, b)
    F = oracle.BSM.of(Fm)
    G = P.BlockSparse.from_host(Fm)
    # no dense spectrum at this size: a constant per-step delta
    p = oracle.SP2Params(n_occ=n // 2, eps=1e-6, taus=synth.tau_log(32), delta_const=1e-9)
    X0o, _, st, _ = oracle.sp2_start(F, p)
    yield n, G, X0o.sorted(), st
    del G


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_sys3d_65536_first_step(sys3d_65536, precision):
    n, G, X0s, st = sys3d_65536
    n_occ, taus = n // 2, synth.tau_log(32)
    prec = P.PRECISIONS[precision]
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, delta_const=1e-9, precision=prec)
    # one step: X^_1 has at most 243k blocks (the pattern of X~_0 squared)
    res = P.purify(G, n_occ, 1e-6, taus, delta_const=1e-9, n_max=1, keep_tape=True, precision=precision,
                   cap=300000)
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    assert len(steps) == 1
    rng = np.random.default_rng(65536 + prec)
    xh, xl = st.xh, st.xl
    for t, lg in enumerate(steps):
        X, nu_g = to_oracle(res.tape(t))
        if t == 0:
            assert np.array_equal(X.keys(), X0s.keys())
            assert np.array_equal(X.vals.view(np.uint64), X0s.vals.view(np.uint64))   # bit for bit
        check_step(X, nu_g, lg, xh, xl, p, res.tape(t + 1), rng)
        if prec:
            assert lg["npairs_low"] > 0
        del X
    del res
    torch.cuda.empty_cache()
