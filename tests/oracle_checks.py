"""Shared checks of GPU purification results against the CPU oracle (a
helper for the GPU tests; collected by no test runner itself).

* end_to_end: an FP64 run equals the oracle's run of the same parameters
  record by record (branch, threshold index and value, kept pairs, delta)
  and in its result (same blocks, values within 1e-12);
* teacher_forced: each step of a run kept on a tape, recomputed by the
  oracle from the GPU's own previous iterate, takes the same decisions
  (branch, tau, sigma, kept and low-tier pairs) -- the check for the
  precision tiers, whose products differ from the oracle's FP64 ones by
  rounding.
"""
import numpy as np

import oracle


def to_oracle(M) -> oracle.BSM:
    brow, bcol, vals, _, _, _ = M.live()
    return oracle.BSM(M.n, M.b, brow, bcol, vals)


PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}


def params(n_occ, taus, homo, lumo, variant="hybrid", precision="fp64", eps=1e-6, **kw):
    return oracle.SP2Params(n_occ=n_occ, eps=eps, taus=taus, homo=homo, lumo=lumo, variant=variant,
                            precision=PREC[precision], **kw)


def end_to_end(Fm, p, logs, D, tol=1e-12):
    """FP64 run (records `logs`, result D on the device) against oracle.sp2."""
    Do, logs_o, _ = oracle.sp2(oracle.BSM.of(Fm), p)
    assert len(logs) == len(logs_o), (len(logs), len(logs_o))
    for lg, lo in zip(logs, logs_o):
        assert lg["branch"] == lo.branch, (lg["i"], lg["branch"], lo.branch)
        if lo.branch >= 0:
            assert lg["idx"] == lo.idx and lg["tau"] == lo.tau, (lg["i"], lg["idx"], lo.idx)
            assert lg["npairs"] == lo.npairs and lg["nout"] == lo.nout, (lg["i"], lg["npairs"], lo.npairs)
            assert lg["delta"] == lo.delta
    Dg = to_oracle(D)
    assert np.array_equal(Dg.keys(), Do.keys())
    assert np.abs(Dg.to_dense() - Do.to_dense()).max() < tol
    return Do


def teacher_forced(Fm, p, res):
    """Every step of a taped run (res.tape(t)) recomputed by oracle.sp2_step
    from the GPU's iterate: same decisions."""
    F = oracle.BSM.of(Fm)
    _, _, st, _ = oracle.sp2_start(F, p)
    xh, xl, e_hist = st.xh, st.xl, []
    steps = [lg for lg in res.logs if lg["branch"] >= 0]
    low = 0
    for t, lg in enumerate(steps):
        Xprev = to_oracle(res.tape(t))
        Xn, _, log, st2 = oracle.sp2_step(Xprev, oracle.SP2State(t + 1, xh, xl, list(e_hist)), p)
        assert Xn is not None
        assert lg["branch"] == log.branch and lg["delta"] == log.delta
        assert lg["idx"] == log.idx and lg["tau"] == log.tau
        assert lg["sidx"] == log.sidx and lg["sigma"] == log.sigma
        assert lg["npairs"] == log.npairs and lg["npairs_low"] == log.npairs_low
        low += lg["npairs_low"]
        xh, xl, e_hist = st2.xh, st2.xl, st2.e_hist
    return low
