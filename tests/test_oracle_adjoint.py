"""Pins of the oracle's reverse mode (frozen kept sets, truncation patterns,
branches and Gerschgorin bounds; not in the paper):

* the frozen replay reproduces the recorded forward run bit for bit;
* one step: the reverse step is the transpose of the step's derivative
  (central differences of a quadratic map are exact up to rounding);
* zero tolerances: the gradient equals the dense chain rule of the SP2
  polynomial (X^2 -> G X + X G, 2X - X^2 -> 2G - G X - X G);
* the whole run: <Fbar, H> against central finite differences of the frozen
  map, on the chain and on a 3D system, with truncation active;
* against the derivative of the exact spectral projector (eigh based,
  approximation-limited) on a small chain."""
import numpy as np
import pytest

import oracle
import synth


def sym_rand_on(P: oracle.BSM, rng) -> oracle.BSM:
    """Random symmetric values on the (symmetric) pattern of P."""
    n = P.nb * P.b
    M = rng.standard_normal((n, n))
    M = M + M.T
    blk = {}
    for t in range(P.nblk):
        r, c = int(P.brow[t]), int(P.bcol[t])
        blk[(r, c)] = M[r * P.b:(r + 1) * P.b, c * P.b:(c + 1) * P.b]
    out = oracle._from_blocks(P, blk)
    # zero the padding past n so H stays a perturbation of the n x n matrix
    for t in range(out.nblk):
        r, c = int(out.brow[t]), int(out.bcol[t])
        rr, cc = min(P.b, P.n - r * P.b), min(P.b, P.n - c * P.b)
        v = out.vals[t].T.copy()
        v[rr:, :] = 0.0
        v[:, cc:] = 0.0
        out.vals[t] = v.T
    return out


def inner(A: oracle.BSM, B: oracle.BSM) -> float:
    """<A, B> over the blocks of A that B also has."""
    bm = B.block_map()
    s = 0.0
    for t in range(A.nblk):
        u = bm[int(A.brow[t]) * A.nb + int(A.bcol[t])]
        if u >= 0:
            s += float(np.sum(A.vals[t] * B.vals[u]))
    return s


def add(A: oracle.BSM, H: oracle.BSM, h: float) -> oracle.BSM:
    """A + h H on A's pattern (H on a sub-pattern)."""
    hm = H.block_map()
    vals = A.vals.copy()
    for t in range(A.nblk):
        u = hm[int(A.brow[t]) * A.nb + int(A.bcol[t])]
        if u >= 0:
            vals[t] = vals[t] + h * H.vals[u]
    return oracle.BSM(A.n, A.b, A.brow.copy(), A.bcol.copy(), vals)


def run_taped(F, n_occ, taus, **kw):
    w = np.linalg.eigvalsh(F.to_dense())
    p = oracle.SP2Params(n_occ=n_occ, eps=1e-6, taus=taus, homo=w[n_occ - 1], lumo=w[n_occ], **kw)
    D, logs, info = oracle.sp2(F, p, keep_tape=True)
    return D, logs, info, p


def test_replay_reproduces_forward():
    F = oracle.BSM.of(synth.chain1d(256, 3, 32))
    D, logs, info, _ = run_taped(F, 128, synth.tau_paper())
    R = oracle.sp2_replay(F, info["tape"], logs, info["lmin"], info["lmax"])
    assert np.array_equal(R.keys(), D.keys())
    assert np.array_equal(R.vals, D.vals)


@pytest.mark.parametrize("branch", [0, 1])
def test_step_is_transpose_of_derivative(branch):
    rng = np.random.default_rng(11 + branch)
    F = oracle.BSM.of(synth.sys3d(384, 4, 32))
    lmin, lmax = oracle.gerschgorin(F)
    X = oracle.x0(F, lmin, lmax)
    C0, _ = oracle.spamm(X, X, 0.0, sym=True)      # a squared iterate: spread of norms
    X = oracle.truncate(C0, 1e-3)[0]
    nu = oracle.norms(X)[1]
    tau = float(np.quantile(nu, 0.3) * np.quantile(nu, 0.5))
    # the forward step with frozen K and the output pattern S'
    K = oracle.kept(X, X, tau, True, nu, nu)
    assert 0 < K.npairs < oracle.kept(X, X, 0.0, True, nu, nu).npairs

    def step(Y):
        V = oracle.block_products(Y, Y, K)
        off = K.oi != K.oj
        C = oracle.BSM(Y.n, Y.b, np.concatenate([K.oi, K.oj[off]]).astype(np.int32),
                       np.concatenate([K.oj, K.oi[off]]).astype(np.int32),
                       np.ascontiguousarray(np.concatenate([V, V[off].transpose(0, 2, 1)]))).sorted()
        return oracle.combine(Y, C, branch).sorted()

    S1 = step(X)
    G = sym_rand_on(S1, rng)
    Xbar = oracle.adjoint_step(X, G, tau, branch, nu)
    H = sym_rand_on(X, rng)
    h = 1e-3
    d = (inner(G, step(add(X, H, h))) - inner(G, step(add(X, H, -h)))) / (2 * h)
    got = inner(Xbar, H)
    assert abs(got - d) <= 1e-10 * (abs(d) + 1.0)
    assert abs(got) > 1e-3           # the check is not vacuous


def test_zero_tolerance_equals_dense_chain_rule():
    rng = np.random.default_rng(5)
    F = oracle.BSM.of(synth.chain1d(192, 5, 32))
    D, logs, info, p = run_taped(F, 96, synth.tau_paper(), delta_const=0.0, n_max=20)
    assert all(l.tau == 0.0 for l in logs if l.branch >= 0)
    n = F.n
    Wm = rng.standard_normal((n, n))
    Wm = Wm + Wm.T
    Dbar = oracle._mask(oracle.from_dense(Wm, F.b), D)
    Fbar = oracle.sp2_adjoint(F, info["tape"], logs, info["lmin"], info["lmax"], Dbar)
    # dense chain rule of the polynomial with the same branch sequence
    lmin, lmax = info["lmin"], info["lmax"]
    Xs = [(lmax * np.eye(n) - F.to_dense()) / (lmax - lmin)]
    steps = [l for l in logs if l.branch >= 0]
    for l in steps:
        X = Xs[-1]
        Xs.append(X @ X if l.branch == 0 else 2 * X - X @ X)
    G = Wm.copy()
    for t in range(len(steps), 0, -1):
        X = Xs[t - 1]
        GX = G @ X + X @ G
        G = GX if steps[t - 1].branch == 0 else 2 * G - GX
    want = -G / (lmax - lmin)
    got = np.zeros((n, n))
    Fd = Fbar.to_dense()
    mask = np.zeros((n, n), dtype=bool)
    for t in range(F.nblk):
        r, c = int(F.brow[t]), int(F.bcol[t])
        mask[r * F.b:(r + 1) * F.b, c * F.b:(c + 1) * F.b] = True
    got[mask] = Fd[mask]
    assert np.linalg.norm(got - want * mask) <= 1e-12 * np.linalg.norm(want * mask)


@pytest.mark.parametrize("case", ["chain", "sys3d"])
def test_adjoint_vs_finite_differences(case):
    rng = np.random.default_rng(21)
    if case == "chain":
        F = oracle.BSM.of(synth.chain1d(256, 7, 32))
        n_occ, taus = 128, synth.tau_paper()
    else:
        F = oracle.BSM.of(synth.sys3d(768, 9, 32))
        n_occ, taus = 384, synth.tau_log(32)
    D, logs, info, _ = run_taped(F, n_occ, taus)
    steps = [l for l in logs if l.branch >= 0]
    assert any(l.tau > 0.0 for l in steps) and any(l.branch == 1 for l in steps)
    assert any(l.trunc is not None and l.trunc.removed_keys.shape[0] > 0 for l in steps)
    Wb = sym_rand_on(D, rng)
    Fbar = oracle.sp2_adjoint(F, info["tape"], logs, info["lmin"], info["lmax"], Wb)
    H = sym_rand_on(F, rng)
    got = inner(Fbar, H)
    lmin, lmax = info["lmin"], info["lmax"]
    h = 1e-6
    Lp = inner(Wb, oracle.sp2_replay(add(F, H, h), info["tape"], logs, lmin, lmax))
    Lm = inner(Wb, oracle.sp2_replay(add(F, H, -h), info["tape"], logs, lmin, lmax))
    fd = (Lp - Lm) / (2 * h)
    assert abs(got - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("tol", ["zero", "eps1e-6"])
def test_adjoint_vs_spectral_projector_derivative(tol):
    """dD[H] of the exact projector onto the n_occ lowest eigenvectors is
    sum over occupied a, virtual v of (u_a^T H u_v)/(e_a - e_v) (u_a u_v^T +
    u_v u_a^T).  With zero tolerances the SP2 polynomial has converged to the
    projector and so has its derivative (tight pin).  With truncation the
    frozen masks drop the paths through removed blocks, which are small in
    value but not in sensitivity: approximation-limited, loose bound."""
    rng = np.random.default_rng(3)
    F = oracle.BSM.of(synth.chain1d(256, 2, 32))
    n = F.n
    n_occ = 128
    kw = dict(delta_const=0.0, n_max=40) if tol == "zero" else {}
    D, logs, info, _ = run_taped(F, n_occ, synth.tau_paper(), **kw)
    Wm = rng.standard_normal((n, n))
    Wm = Wm + Wm.T
    Wb = oracle._mask(oracle.from_dense(Wm, F.b), D)
    Fbar = oracle.sp2_adjoint(F, info["tape"], logs, info["lmin"], info["lmax"], Wb)
    e, U = np.linalg.eigh(F.to_dense())
    Wt = U.T @ Wb.to_dense() @ U
    occ = np.arange(n) < n_occ
    Gam = np.zeros((n, n))
    de = e[:, None] - e[None, :]
    cross = occ[:, None] != occ[None, :]
    Gam[cross] = (occ[:, None].astype(float) - occ[None, :].astype(float))[cross] / de[cross]
    Fex = U @ (Gam * Wt) @ U.T
    mask = np.zeros((n, n), dtype=bool)
    for t in range(F.nblk):
        r, c = int(F.brow[t]), int(F.bcol[t])
        mask[r * F.b:(r + 1) * F.b, c * F.b:(c + 1) * F.b] = True
    rel = np.linalg.norm((Fbar.to_dense() - Fex)[mask]) / np.linalg.norm(Fex[mask])
    assert rel < (1e-10 if tol == "zero" else 1e-2)
