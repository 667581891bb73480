"""Small systems (nb <= 64): the single-workgroup passes (occupancy and the
sweep's cube list, kept pairs and output pattern, truncation) against the
device-wide passes on the same inputs.  Both build the same lists in the
same order, so every per-iteration record and the result are bit-identical
with the switch on and off: FP64 and both tiers, Algorithm 3's bound and
B_flat, the three variants, the host-driven and the graph-captured loop,
the batched driver, and the product / truncation entry points on their own
(non-symmetric operands, ragged nb, a matrix with empty rows).  The oracle
comparisons of the other GPU tests run with the switch on (the default)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2005_10680_amd as P  # noqa: E402

FIELDS = ["i", "branch", "idx", "stop", "delta", "tau", "t1", "t2", "e", "npairs", "nout", "nslot_hat",
          "nslot_kept", "removed_units", "removed_fro2", "npairs_low", "sigma", "sidx"]


@pytest.fixture
def both_paths():
    """Runs f with the small-system passes on and off, restores the default."""
    def run(f):
        try:
            P.set_small_path(True)
            a = f()
            P.set_small_path(False)
            b = f()
        finally:
            P.set_small_path(True)
        return a, b
    return run


def same_logs(la, lb):
    assert len(la) == len(lb)
    for a, b in zip(la, lb):
        for f in FIELDS:
            assert a[f] == b[f], (f, a["i"], a[f], b[f])


def same_matrix(A, B, norms=True):
    b1, c1, v1, n1, s1, _ = A.live()
    b2, c2, v2, n2, s2, _ = B.live()
    assert np.array_equal(b1, b2) and np.array_equal(c1, c2)
    assert np.array_equal(v1.view(np.uint64), v2.view(np.uint64))
    if not norms:  # the product entry points leave C's norms to spamm_build_norms
        return
    assert np.array_equal(n1.view(np.uint64), n2.view(np.uint64))
    assert np.array_equal(s1.view(np.uint64), s2.view(np.uint64))


def system(kind, n, b, seed):
    Fm = synth.chain1d(n, seed, b) if kind == "chain" else synth.sys3d(n, seed, b)
    w = np.linalg.eigvalsh(oracle.BSM.of(Fm).to_dense())
    taus = synth.tau_paper() if kind == "chain" else synth.tau_log(32)
    return Fm, n // 2, taus, w[n // 2 - 1], w[n // 2]


@pytest.mark.parametrize("kind,n,b,seed,variant,precision,bound,graph", [
    ("chain", 1024, 32, 1, "hybrid", "fp64", "tree", 0),
    ("chain", 1024, 32, 1, "hybrid", "fp64", "tree", 8),
    ("chain", 1024, 32, 1, "spamm", "fp64", "tree", 0),
    ("chain", 1024, 32, 1, "truncmul", "fp64", "tree", 8),
    ("sys3d", 2000, 64, 5, "hybrid", "fp64", "tree", 0),
    ("sys3d", 2000, 64, 5, "hybrid", "fp32", "tree", 4),
    ("sys3d", 1500, 32, 6, "hybrid", "bf16x3", "tree", 0),      # nb = 47 (ragged)
    ("sys3d", 1500, 32, 6, "hybrid", "fp64", "flat", 0),
    ("sys3d", 2048, 32, 7, "hybrid", "fp32", "flat", 8),       # nb = 64, the largest small system
])
def test_purify_small_path_bit_identical(both_paths, kind, n, b, seed, variant, precision, bound, graph):
    Fm, n_occ, taus, homo, lumo = system(kind, n, b, seed)
    F = P.BlockSparse.from_host(Fm)
    assert F.nb <= 64
    r1, r2 = both_paths(lambda: P.purify(F, n_occ, 1e-6, taus, homo=homo, lumo=lumo, variant=variant,
                                         precision=precision, bound=bound, graph_steps=graph))
    assert r1.status == r2.status
    same_logs(r1.logs, r2.logs)
    same_matrix(r1.D, r2.D)
    assert sum(1 for lg in r1.logs if lg["branch"] >= 0) >= 5


def test_batched_small_path_bit_identical(both_paths):
    mats = [system("chain", 1024, 32, 1), system("sys3d", 1000, 64, 11), system("sys3d", 4096, 64, 12)]
    Fs = [P.BlockSparse.from_host(m[0]) for m in mats]            # nb 32, 16 and 64
    kw = dict(n_occ=[m[1] for m in mats], taus=[m[2] for m in mats], homo=[m[3] for m in mats],
              lumo=[m[4] for m in mats])
    r1, r2 = both_paths(lambda: P.purify_batched(Fs, eps=1e-6, precision=["fp64", "fp32", "bf16x3"], **kw))
    for q in range(len(Fs)):
        same_logs(r1.logs[q], r2.logs[q])
        same_matrix(r1.D[q], r2.D[q])


def test_multiply_and_truncate_small_path(both_paths):
    """spamm_multiply on non-symmetric operands (general and transposed B
    layout, an all-empty block row in A), then spamm_truncate of a symmetric
    product: same pattern, values, kept counts and removed units."""
    rng = np.random.default_rng(3)
    n, b = 1400, 32                                   # nb = 44
    A = synth.sys3d(n, 21, b)
    B = synth.sys3d(n, 22, b)
    Am = oracle.BSM.of(A)
    keep = Am.brow != 3                               # block row 3 of A empty
    Am = oracle.BSM(Am.n, Am.b, Am.brow[keep], Am.bcol[keep], Am.vals[keep])
    dA, dB = P.BlockSparse.from_host(Am), P.BlockSparse.from_host(B)
    P.build_norms(dA)
    P.build_norms(dB)
    nuA = oracle.norms(Am)[1]
    tau = float(np.quantile(nuA, 0.4)) * float(np.quantile(oracle.norms(oracle.BSM.of(B))[1], 0.4))
    for bt in (False, True):
        (C1, k1), (C2, k2) = both_paths(lambda: P.multiply(dA, dB, tau, b_transposed=bt))
        torch.cuda.synchronize()
        assert torch.equal(k1, k2) and int(k1[0]) > 0
        same_matrix(C1, C2, norms=False)
    R = rng.standard_normal((n, n)) * 1e-3
    i = np.arange(n)
    R *= np.exp(-np.abs(i[:, None] - i[None, :]) / 60.0)   # decaying blocks: some fall below delta
    S = P.BlockSparse.from_host(oracle.from_dense(R + R.T, b))
    P.build_norms(S)
    (C1, _), (C2, _) = both_paths(lambda: P.multiply(S, S, 0.0, symmetric=True, b_transposed=True,
                                                         max_pairs=S.nb ** 3))
    same_matrix(C1, C2, norms=False)
    fro = float(np.sqrt(np.sum(oracle.norms(oracle.BSM(C1.n, C1.b, *C1.live()[:3]))[0])))
    for delta in (1e-3 * fro, 0.1 * fro):
        def trunc():
            X = P.BlockSparse.from_host(oracle.BSM(C1.n, C1.b, *C1.live()[:3]))
            P.build_norms(X)
            rem = P.truncate(X, delta, sync=True)
            return X, rem.cpu().numpy()
        (X1, r1), (X2, r2) = both_paths(trunc)
        assert np.array_equal(r1, r2) and r1[0] > 0
        same_matrix(X1, X2)
