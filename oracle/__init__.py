"""CPU FP64 oracle for SpAMM with error control inside SP2 purification.

TEST INFRASTRUCTURE ONLY: the plain, slow, obviously-correct reference the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; the product path
(``paper_2005_10680_amd``) never does, and the two share no code.

Heavy loops live in ``oracle.c`` (plain C, one IEEE operation per source
operation); this module does the orchestration in numpy.  Every function
names the part of the paper it follows.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  norms          exact rounding pinned to math.fsum of exact square splits
  cse_tree       pinned to the worked example, eqs. (3)-(6), to the closed
                 form at nb = 2, to brute force and to bound orderings
  kept / spamm   pinned to brute force and to the dense product at tau = 0
  truncate       pinned to direct recomputation of ||E||_F and maximality
  sp2            pinned to diagonal F (exact step function) and to dense
                 eigendecomposition on small systems
  adjoint        pinned to finite differences and to the Frechet derivative
                 of the step function (eigh-based) on small systems
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, d = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.o_block_sq.argtypes = [P, i64, P, P]
        L.o_norms.argtypes = [i64, i32, P, P, P]
        L.o_exact_sum_nonneg.argtypes = [P, i64]
        L.o_exact_sum_nonneg.restype = d
        L.o_cse_tree.argtypes = [i32, P, P, P, P, P, i32, i32, d, d, P]
        L.o_cse_tree.restype = i32
        L.o_cse_tree_leafvals.argtypes = [i32, P, P, P, P]
        L.o_cse_tree_leafvals.restype = i32
        L.o_cse_flat_sum.argtypes = [i32, P, P, P, P, P, i32, i32, d, d, P, P]
        L.o_kept_counts.argtypes = [i32, P, P, P, P, d, i32, P]
        L.o_kept_lists.argtypes = [i32, P, P, P, P, d, i64, P, P, P, P]
        L.o_block_products.argtypes = [i32, i32, P, P, P, P, i64, P, P, P, P, P]
        L.o_traces.argtypes = [i64, i32, i64, P, P, P, P]
        L.o_gerschgorin.argtypes = [i64, i32, i64, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Block-sparse container (the oracle's own; independent of the GPU library)
# ---------------------------------------------------------------------------

@dataclass
class BSM:
    """Block-sparse matrix: blocks (brow[k], bcol[k]) with vals[k, col, row]."""
    n: int
    b: int
    brow: np.ndarray
    bcol: np.ndarray
    vals: np.ndarray
    _map: np.ndarray | None = field(default=None, repr=False)

    @property
    def nb(self):
        return (self.n + self.b - 1) // self.b

    @property
    def nblk(self):
        return int(self.brow.shape[0])

    @staticmethod
    def of(M) -> "BSM":
        """From any object with n, b, brow, bcol, vals (e.g. synth.BlockMatrix)."""
        return BSM(int(M.n), int(M.b), np.ascontiguousarray(M.brow, dtype=np.int32),
                   np.ascontiguousarray(M.bcol, dtype=np.int32),
                   np.ascontiguousarray(M.vals, dtype=np.float64))

    def block_map(self) -> np.ndarray:
        """map[r*nb + c] = index of block (r, c) or -1 (an absent quadrant)."""
        if self._map is None:
            m = np.full(self.nb * self.nb, -1, dtype=np.int32)
            m[self.brow.astype(np.int64) * self.nb + self.bcol] = np.arange(self.nblk, dtype=np.int32)
            self._map = m
        return self._map

    def to_dense(self) -> np.ndarray:
        nb, b = self.nb, self.b
        D = np.zeros((nb * b, nb * b))
        for k in range(self.nblk):
            r, c = int(self.brow[k]), int(self.bcol[k])
            D[r * b:(r + 1) * b, c * b:(c + 1) * b] = self.vals[k].T
        return D[: self.n, : self.n]

    def keys(self) -> np.ndarray:
        return self.brow.astype(np.int64) * self.nb + self.bcol

    def subset(self, keep: np.ndarray) -> "BSM":
        return BSM(self.n, self.b, self.brow[keep].copy(), self.bcol[keep].copy(),
                   np.ascontiguousarray(self.vals[keep]))

    def sorted(self) -> "BSM":
        o = np.argsort(self.keys(), kind="stable")
        return self.subset(o)


def from_dense(D: np.ndarray, b: int) -> BSM:
    n = D.shape[0]
    nb = (n + b - 1) // b
    P = np.zeros((nb * b, nb * b))
    P[:n, :n] = D
    T = P.reshape(nb, b, nb, b).transpose(0, 2, 3, 1)
    present = np.any(T != 0.0, axis=(2, 3))
    rr, cc = np.nonzero(present)
    return BSM(n, b, rr.astype(np.int32), cc.astype(np.int32), np.ascontiguousarray(T[rr, cc]))


# ---------------------------------------------------------------------------
# Norms (skip test of Algorithm 2, leaf values of Algorithm 3)
# ---------------------------------------------------------------------------

def norms(X: BSM):
    """(sq, nu): sq = RN(exact sum of squares) per block, nu = sqrt_RN(sq)."""
    sq = np.empty(X.nblk)
    nu = np.empty(X.nblk)
    if X.nblk:
        lib().o_norms(X.nblk, X.b, _p(X.vals), _p(sq), _p(nu))
    return sq, nu


# ---------------------------------------------------------------------------
# Algorithm 3 (CSE) and the selection rule that follows it
# ---------------------------------------------------------------------------

def cse_tree(A: BSM, B: BSM, taus, nuA=None, nuB=None, mode=0, tau0=0.0, c_low=0.0) -> np.ndarray:
    """Error bound of SpAMM(A, B, tau_k) for every candidate (Algorithm 3)."""
    taus = np.ascontiguousarray(taus, dtype=np.float64)
    if nuA is None:
        nuA = norms(A)[1]
    if nuB is None:
        nuB = norms(B)[1]
    nuA = np.ascontiguousarray(nuA, dtype=np.float64)
    nuB = np.ascontiguousarray(nuB, dtype=np.float64)
    out = np.zeros(taus.shape[0])
    rc = lib().o_cse_tree(A.nb, _p(A.block_map()), _p(nuA), _p(B.block_map()), _p(nuB), _p(taus),
                          taus.shape[0], mode, tau0, c_low, _p(out))
    assert rc == 0
    return out


def cse_tree_leafvals(A: BSM, B: BSM, leafvals: np.ndarray) -> float:
    """Algorithm 3's combination rule on explicit leaf errors
    leafvals[i, k, j] (0 where the product is kept)."""
    lv = np.ascontiguousarray(leafvals, dtype=np.float64)
    assert lv.shape == (A.nb, A.nb, A.nb)
    out = np.zeros(1)
    rc = lib().o_cse_tree_leafvals(A.nb, _p(A.block_map()), _p(B.block_map()), _p(lv), _p(out))
    assert rc == 0
    return float(out[0])


def cse_flat_sum(A: BSM, B: BSM, taus, nuA=None, nuB=None, mode=0, tau0=0.0, c_low=0.0):
    """Leaf-level bounds for every candidate: B_flat = (sum over outputs of
    (sum over k of the leaf values)^2)^(1/2) (eq. (6) applied to each output's
    leaf blocks) and B_sum = the sum of all leaf values.  Leaf values as in
    Algorithm 3: p when p < tau_k (mode 0); in mode 1 (precision tiers) p when
    p < tau0, c_low p when tau0 <= p < tau_k, else 0.  Per output the leaf
    values are summed in ascending k (one rounding per addition), s_ij; the
    sums over outputs are exact, rounded once: B_sum = RN(sum s_ij),
    B_flat = sqrt_RN(RN(sum RN(s_ij^2))), independent of the output order."""
    taus = np.ascontiguousarray(taus, dtype=np.float64)
    nuA = norms(A)[1] if nuA is None else np.ascontiguousarray(nuA)
    nuB = norms(B)[1] if nuB is None else np.ascontiguousarray(nuB)
    flat = np.zeros(taus.shape[0])
    ssum = np.zeros(taus.shape[0])
    lib().o_cse_flat_sum(A.nb, _p(A.block_map()), _p(nuA), _p(B.block_map()), _p(nuB), _p(taus),
                         taus.shape[0], int(mode), float(tau0), float(c_low), _p(flat), _p(ssum))
    return flat, ssum


def select(bound: np.ndarray, taus: np.ndarray, budget: float):
    """Pick the candidate whose bound is the largest one below the budget.
    Bounds do not increase along the (decreasing) candidate list, so this is
    the first m with bound_m < budget; none -> (N, 0.0): exact product."""
    for m in range(len(bound)):
        if bound[m] < budget:
            return m, float(taus[m])
    return len(bound), 0.0


# ---------------------------------------------------------------------------
# Algorithm 2 (SpAMM) at the leaf level
# ---------------------------------------------------------------------------

@dataclass
class Kept:
    oi: np.ndarray     # output block rows
    oj: np.ndarray     # output block cols
    kptr: np.ndarray   # int64 [nout+1]
    klist: np.ndarray  # int32 kept inner block indices, ascending per output

    @property
    def npairs(self):
        return int(self.kptr[-1])


def kept(A: BSM, B: BSM, tau: float, sym: bool, nuA=None, nuB=None) -> Kept:
    """Kept triples {(i,k,j): RN(nu(A_ik) nu(B_kj)) >= tau}; outputs in
    row-major order, restricted to i <= j when sym."""
    nuA = norms(A)[1] if nuA is None else np.ascontiguousarray(nuA)
    nuB = norms(B)[1] if nuB is None else np.ascontiguousarray(nuB)
    nb = A.nb
    counts = np.zeros(nb * nb, dtype=np.int32)
    L = lib()
    L.o_kept_counts(nb, _p(A.block_map()), _p(nuA), _p(B.block_map()), _p(nuB), float(tau), int(sym),
                    _p(counts))
    nz = np.nonzero(counts)[0]
    oi = (nz // nb).astype(np.int32)
    oj = (nz % nb).astype(np.int32)
    kptr = np.zeros(nz.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts[nz], out=kptr[1:])
    klist = np.zeros(int(kptr[-1]), dtype=np.int32)
    if nz.shape[0]:
        L.o_kept_lists(nb, _p(A.block_map()), _p(nuA), _p(B.block_map()), _p(nuB), float(tau),
                       nz.shape[0], _p(oi), _p(oj), _p(kptr), _p(klist))
    return Kept(oi, oj, kptr, klist)


def block_products(A: BSM, B: BSM, K: Kept, sel=None) -> np.ndarray:
    """Values of the output blocks of K (or of the outputs listed in sel):
    C_ij = sum over kept k ascending of the textbook product A_ik B_kj."""
    if sel is None:
        oi, oj, kptr, klist = K.oi, K.oj, K.kptr, K.klist
    else:
        sel = np.asarray(sel, dtype=np.int64)
        oi, oj = K.oi[sel], K.oj[sel]
        lens = K.kptr[sel + 1] - K.kptr[sel]
        kptr = np.zeros(sel.shape[0] + 1, dtype=np.int64)
        np.cumsum(lens, out=kptr[1:])
        klist = np.concatenate([K.klist[K.kptr[s]:K.kptr[s + 1]] for s in sel]) if sel.shape[0] else \
            np.zeros(0, dtype=np.int32)
        klist = np.ascontiguousarray(klist, dtype=np.int32)
        oi = np.ascontiguousarray(oi); oj = np.ascontiguousarray(oj)
    b = A.b
    out = np.zeros((oi.shape[0], b, b))
    if oi.shape[0]:
        lib().o_block_products(b, A.nb, _p(A.block_map()), _p(A.vals), _p(B.block_map()), _p(B.vals),
                               oi.shape[0], _p(oi), _p(oj), _p(kptr), _p(klist), _p(out))
    return out


def spamm(A: BSM, B: BSM, tau: float, sym: bool = False, nuA=None, nuB=None):
    """C~ = SpAMM(A, B, tau) (Algorithm 2) on the pattern of the kept
    outputs.  sym: A = B = X symmetric, compute i <= j and mirror
    C~_ji = C~_ij^T.  Returns (C~, Kept)."""
    K = kept(A, B, tau, sym, nuA, nuB)
    V = block_products(A, B, K)
    if sym:
        off = K.oi != K.oj
        brow = np.concatenate([K.oi, K.oj[off]])
        bcol = np.concatenate([K.oj, K.oi[off]])
        vals = np.concatenate([V, V[off].transpose(0, 2, 1)])
    else:
        brow, bcol, vals = K.oi, K.oj, V
    C = BSM(A.n, A.b, brow.astype(np.int32), bcol.astype(np.int32), np.ascontiguousarray(vals)).sorted()
    return C, K


# ---------------------------------------------------------------------------
# Truncation, ||E||_F < delta (Algorithm 1/5 truncation lines)
# ---------------------------------------------------------------------------

KEY_BITS = 40  # quantum Q = 2^(e_T - KEY_BITS), T = RN(delta^2) in [2^e_T, 2^(e_T+1))
KSAT = 1 << 41


@dataclass
class TruncInfo:
    removed_keys: np.ndarray   # upper-block keys r*nb+c (r <= c) of removed units
    removed_fro2: float        # sum of w*sq over removed units (double)
    kt: int                    # integer budget K_T
    ksum: int                  # integer sum of removed keys


def trunc_quanta(delta: float):
    """(T, Q, K_T) of the truncation rule for budget delta: T = RN(delta^2),
    Q = 2^(e_T - 40) with T in [2^e_T, 2^(e_T + 1)) (not below 2^-1000),
    K_T = floor(T/Q).

    Why removing units whose integer keys k = ceil(w sq / Q) sum to less
    than K_T keeps ||E||_F < delta: the key sum is then at most K_T - 1, so
    sum(w sq) <= Q (K_T - 1) <= T - Q; Q > 2^-41 T, and each sq is the
    exact sum of squares S rounded once (S <= sq (1 + 2^-52)), so the exact
    removed sum of squares is below (T - Q)(1 + 2^-52) < T (1 - 2^-42) and
    T <= delta^2 (1 + 2^-53): below delta^2.  With a key sum equal to K_T
    it could reach T, which may exceed delta^2 when RN rounded up."""
    T = delta * delta
    if not (T > 0.0 and math.isfinite(T)):
        return T, 0.0, 0
    e_T = math.frexp(T)[1] - 1
    Q = math.ldexp(1.0, max(e_T - KEY_BITS, -1000))
    kt = int(math.floor(T / Q))
    return T, Q, kt


def trunc_keys(sq_upper: np.ndarray, w: np.ndarray, Q: float) -> np.ndarray:
    """k_u = ceil(w*sq/Q), saturated at 2^41 (exact integers)."""
    v = w * sq_upper
    with np.errstate(over="ignore", invalid="ignore"):
        s = v / Q
    k = np.where(s < float(KSAT), np.ceil(np.where(s < float(KSAT), s, 0.0)), float(KSAT))
    return k.astype(np.uint64)


def truncate(X: BSM, delta: float, sq=None):
    """Remove whole symmetric units (diagonal blocks; off-diagonal pairs) in
    ascending order of their quantised squared norm, ties by coordinates,
    as long as the removed squared Frobenius norm provably stays below
    delta^2.  Returns (X~, TruncInfo)."""
    if sq is None:
        sq = norms(X)[0]
    nb = X.nb
    up = X.brow <= X.bcol
    ukeys = X.keys()[up]
    sq_up = sq[up]
    w = np.where(X.brow[up] == X.bcol[up], 1.0, 2.0)
    T, Q, kt = trunc_quanta(delta)
    if kt <= 0:
        return X, TruncInfo(np.zeros(0, dtype=np.int64), 0.0, kt, 0)
    k = trunc_keys(sq_up, w, Q)
    order = np.lexsort((ukeys, k))
    csum = np.cumsum(k[order], dtype=np.uint64)  # exact: < 2^22 units * 2^41
    q = int(np.searchsorted(csum, np.uint64(kt), side="left"))  # first index with csum >= kt
    removed = ukeys[order[:q]]
    ksum = int(csum[q - 1]) if q else 0
    fro2 = float(np.sum((w * sq_up)[order[:q]])) if q else 0.0
    rem_r, rem_c = removed // nb, removed % nb
    drop = np.zeros(nb * nb, dtype=bool)
    drop[removed] = True
    drop[rem_c * nb + rem_r] = True
    keep = ~drop[X.keys()]
    return X.subset(keep), TruncInfo(np.sort(removed), fro2, kt, ksum)


# ---------------------------------------------------------------------------
# Purification pieces: starting matrix, traces, SP2 (Algorithms 1, 4, 5)
# ---------------------------------------------------------------------------

def gerschgorin(F: BSM):
    out = np.zeros(2)
    lib().o_gerschgorin(F.nblk, F.b, F.n, _p(F.brow), _p(F.bcol), _p(F.vals), _p(out))
    return float(out[0]), float(out[1])


def x0(F: BSM, lmin: float, lmax: float) -> BSM:
    """X_0 = (lmax I - F) / (lmax - lmin): the linear map of F sending its
    spectrum into [0, 1], occupied states near 1 (the starting matrix of the
    purification algorithms).  Entry-wise, with W = RN(lmax - lmin):
    diagonal x = RN(RN(lmax - f) / W), off-diagonal x = RN(-f / W); padding
    past n is +0.  Every diagonal block is present."""
    nb, b, n = F.nb, F.b, F.n
    W = lmax - lmin
    M = F.block_map()
    dmiss = [d for d in range(nb) if M[d * nb + d] < 0]
    brow = np.concatenate([F.brow, np.array(dmiss, dtype=np.int32)])
    bcol = np.concatenate([F.bcol, np.array(dmiss, dtype=np.int32)])
    vals = np.concatenate([F.vals, np.zeros((len(dmiss), b, b))])
    ar = np.arange(b)
    gi = brow[:, None, None].astype(np.int64) * b + ar[None, None, :]   # row of vals[k, col, row]
    gj = bcol[:, None, None].astype(np.int64) * b + ar[None, :, None]   # col
    on_diag = gi == gj
    out = np.where(on_diag, (lmax - vals) / W, (-vals) / W)
    out = np.where((gi < n) & (gj < n), out, 0.0)
    return BSM(n, b, brow, bcol, np.ascontiguousarray(out)).sorted()


def traces(X: BSM):
    """(t1, t2, e) = RN(tr X), RN(||X||_F^2), RN(tr X - ||X||_F^2), exact sums."""
    out = np.zeros(3)
    lib().o_traces(X.nblk, X.b, X.n, _p(X.brow), _p(X.bcol), _p(X.vals), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def combine(X: BSM, C: BSM, branch: int) -> BSM:
    """X^ = C (branch 0, f(x) = x^2) or RN(RN(2x) - c) (branch 1, f(x) = 2x - x^2)
    on the union pattern."""
    if branch == 0:
        return C
    nb = X.nb
    keys = np.union1d(X.keys(), C.keys())
    b = X.b
    vals = np.zeros((keys.shape[0], b, b))
    xm = {int(k): i for i, k in enumerate(X.keys())}
    cm = {int(k): i for i, k in enumerate(C.keys())}
    for t, kk in enumerate(keys):
        kk = int(kk)
        xv = 2.0 * X.vals[xm[kk]] if kk in xm else np.zeros((b, b))
        if kk in cm:
            xv = xv - C.vals[cm[kk]]
        vals[t] = xv
    return BSM(X.n, b, (keys // nb).astype(np.int32), (keys % nb).astype(np.int32), vals)


# the FP32 tier evaluates a pair only when both of its blocks have a norm of
# at least this (see tier_constant): below it the pair stays FP64
FP32_TIER_NORM_MIN = 2.0 ** -40


def low_tier_pairs(X: "BSM", tau: float, sigma: float, nu: np.ndarray, precision: int) -> int:
    """Kept pairs of the symmetric product X X evaluated in the low tier:
    tau <= p < sigma, and for the FP32 tier both block norms at least
    FP32_TIER_NORM_MIN."""
    if not sigma > tau:
        return 0
    K = kept(X, X, tau, True, nu, nu)
    if K.npairs == 0:
        return 0
    nb = X.nb
    mp = X.block_map()
    counts = (K.kptr[1:] - K.kptr[:-1]).astype(np.int64)
    ii = np.repeat(K.oi.astype(np.int64), counts)
    jj = np.repeat(K.oj.astype(np.int64), counts)
    kk = K.klist.astype(np.int64)
    na = nu[mp[ii * nb + kk]]
    nbv = nu[mp[kk * nb + jj]]
    p = na * nbv
    low = p < sigma
    if precision == 1:
        low &= (na >= FP32_TIER_NORM_MIN) & (nbv >= FP32_TIER_NORM_MIN)
    return int(np.count_nonzero(low))


def tier_constant(precision: int, b: int) -> float:
    """Per-pair rounding factor c of a low-precision leaf-product tier (not in
    the paper): ||fl(AB) - AB||_F <= c ||A||_F ||B||_F for one b x b pair.

    precision 1, FP32: operands rounded to FP32 (unit roundoff u = 2^-24
    each), b products accumulated in FP32 with an assumed unit roundoff of
    2u: |fl(AB) - AB| <= (2u + u^2 + gamma_b(2u) (1+u)^2) |A||B| entrywise,
    gamma_m(x) = m x / (1 - m x), then Cauchy-Schwarz per entry.  Entries
    and partial results below FP32's normal range (2^-126) may lose up to
    2^-126 each (flushed to zero): with both blocks' norms at least
    FP32_TIER_NORM_MIN = 2^-40 (the tier takes no other pair) that adds at
    most b^2 2^-126 / 2^-80 + 2 b 2^-126 / 2^-40 < 2^-31 relative to
    ||A|| ||B|| for b <= 128, the term "underflow".

    precision 2, split BF16: each block scaled by a power of two (max entry
    in [1, 2)), split x = hi + lo + e with hi = RN_bf16(x), lo = RN_bf16(x -
    hi) (unit roundoff u = 2^-8): |lo| <= u (1+u) |x|, |e| <= u^2 (1+u) |x|;
    the three products hi*hi + hi*lo + lo*hi are exact in FP32 and their 3b
    terms are accumulated in FP32 (unit roundoff 2 * 2^-24 assumed).  The
    dropped terms lo*lo, e*(hi + lo), (hi + lo)*e', e*e' give
    kappa = u^2 ((1+u)^2 + 2 (1+u)^3 + u^2 (1+u)^2), the accumulation
    gamma_3b(2^-23) (1 + 2u)(1+u)^2, and 2^-100 covers entries below the
    BF16 normal range (relative to the scaled blocks, whose norms are >= 1).

    Both rounded up by a factor 1 + 2^-40 (tier_constant_parts gives the
    terms before that factor)."""
    parts = tier_constant_parts(precision, b)
    if not parts:
        return 0.0
    return (parts["represent"] + parts["accumulate"] + parts["underflow"]) * (1.0 + 2.0 ** -40)


def tier_constant_parts(precision: int, b: int) -> dict:
    """The terms of tier_constant (see there), by the error they cover:
    "represent": rounding the operands to the tier's format (FP32: 2u + u^2;
    split BF16: kappa, the dropped lo*lo term and the split residuals);
    "accumulate": the FP32 accumulation of the exact operand products, the
    number of terms per output entry (b for FP32, 3b for the three split
    products) times the assumed unit roundoff 2^-23, as gamma_m, scaled by
    the operands' size relative to the exact ones; "underflow": entries below
    the BF16 normal range (split BF16 only)."""
    m = float(b)
    if precision == 1:
        u = 2.0 ** -24
        ue = 2.0 * u
        gam = m * ue / (1.0 - m * ue)
        return {"represent": 2.0 * u + u * u, "accumulate": gam * (1.0 + u) * (1.0 + u), "underflow": 2.0 ** -31}
    if precision == 2:
        u = 2.0 ** -8
        ue = 2.0 * 2.0 ** -24
        kappa = u * u * ((1.0 + u) ** 2 + 2.0 * (1.0 + u) ** 3 + u * u * (1.0 + u) ** 2)
        gam = 3.0 * m * ue / (1.0 - 3.0 * m * ue)
        return {"represent": kappa, "accumulate": gam * (1.0 + 2.0 * u) * (1.0 + u) ** 2, "underflow": 2.0 ** -100}
    return {}


@dataclass
class SP2Params:
    n_occ: int
    eps: float = 1e-6
    taus: np.ndarray | None = None
    homo: float = float("nan")    # highest occupied eigenvalue of F (or an upper bound)
    lumo: float = float("nan")    # lowest unoccupied eigenvalue of F (or a lower bound)
    n_max: int = 60
    variant: str = "hybrid"       # "hybrid" (Alg. 5), "spamm" (Alg. 4), "truncmul" (Alg. 1)
    delta_const: float = float("nan")  # explicit per-step delta when no gap is given
    e_tol: float = 0.0
    precision: int = 0            # 1: FP32 tier, 2: split-BF16 tier, for tau <= p < sigma (rounding folded into the bound)
    tier_split: float = 0.5       # share of the product budget given to skipping when tiered
    bound: str = "tree"           # "tree": Algorithm 3's recursive bound; "flat" / "sum": leaf-level eq. (6) / plain sum


@dataclass
class SP2State:
    """Everything step i needs besides X~_{i-1}."""
    i: int
    xh: float
    xl: float
    e_hist: list


# RN(2 sqrt(2)): the Davis-Kahan factor of the tolerance schedule
DK_FACTOR = 2.8284271247461903


def step_delta(p: SP2Params, gap: float) -> float:
    """delta_i = eps g_i / (2 sqrt(2) (n_max + 1)), g_i the mapped gap of
    X_i, or the constant.

    Derivation (the paper defers the schedule to the references it cites):
    step i perturbs f_i(X~_{i-1}) by less than delta_i in Frobenius norm
    (SpAMM and truncation together).  With g_i the gap of the exactly mapped
    spectrum around the occupied/virtual split, the Davis-Kahan sin-theta
    theorem moves the projector onto the occupied subspace by at most
    sqrt(2) delta_i / g_i (first order in delta_i / g_i).  A run has at most
    n_max + 1 perturbations (X~_0 and n_max steps), so the projector drifts
    by at most sum sqrt(2) delta_i / g_i <= eps / 2 in all; the other half
    of eps is left to the distance of D~ from its own projector at the
    stop, 2 |tr X~ - ||X~||_F^2| (bounded when the spectrum lies in [0, 1])."""
    if math.isfinite(p.delta_const):
        return p.delta_const
    return p.eps * gap / (DK_FACTOR * float(p.n_max + 1))


def choose_branch(t1: float, t2: float, n_occ: int) -> int:
    """SP2 polynomial for this step: 0 -> x^2, 1 -> 2x - x^2, whichever
    trace lands closer to the occupation (ties -> x^2)."""
    return 0 if abs(t2 - n_occ) <= abs((2.0 * t1 - t2) - n_occ) else 1


def map_gap(x: float, branch: int) -> float:
    return x * x if branch == 0 else 2.0 * x - x * x


def should_stop(e_hist: list, e_tol: float) -> bool:
    """Stop when |e_i| <= e_tol, or when two steps failed to converge
    quadratically: |e_{i-2}| <= 1/8 and |e_i| > 4 e_{i-2}^2 / (1 - 2|e_{i-2}|)^2.

    Derivation (the idea of the parameterless stopping criteria the paper
    cites): e = tr X - ||X||_F^2 = sum_k d_k (1 - d_k) with d_k the distance
    of eigenvalue k to {0, 1}.  Two SP2 steps with different polynomials take
    every d to at most 4 d^2, and for e <= 1/8 every d_k <= 2e, so
    sum d_k <= e / (1 - 2e) and the next e is at most
    4 sum d_k^2 <= 4 e^2 / (1 - 2e)^2 (< e).  Two steps with the same
    polynomial are chosen by the trace rule only when the side they do not
    square is already of second order, which gives the same bound to first
    order.  In exact arithmetic the test therefore never fires; when it does,
    the rounding, SpAMM and truncation errors dominate e and further steps
    add error without convergence.  1/8 is where the bound is a contraction
    (4e / (1 - 2e)^2 < 1 needs e < 0.134)."""
    if not e_hist:
        return False
    if abs(e_hist[-1]) <= e_tol:
        return True
    if len(e_hist) >= 3:
        a = abs(e_hist[-3])
        if a <= 0.125:
            d = 1.0 - 2.0 * a
            if abs(e_hist[-1]) > 4.0 * a * a / (d * d):
                return True
    return False


@dataclass
class StepLog:
    i: int
    branch: int
    delta: float
    bound: np.ndarray
    idx: int
    tau: float
    npairs: int
    nout: int
    trunc: TruncInfo | None
    t1: float
    t2: float
    e: float
    sidx: int = -1
    sigma: float = 0.0
    npairs_low: int = 0


def sp2_step(X: BSM, st: SP2State, p: SP2Params):
    """One iteration of Algorithm 5 (hybrid) / 4 (spamm) / 1 (truncmul) on
    X~_{i-1} = X.  Returns (X~_i, Xhat_i, StepLog, new state) or
    (None, None, log, state) when the stop rule fires before the step."""
    t1, t2, e = traces(X)
    e_hist = st.e_hist + [e]
    if should_stop(e_hist, p.e_tol) or st.i > p.n_max:
        return None, None, StepLog(st.i, -1, 0.0, np.zeros(0), -1, 0.0, 0, 0, None, t1, t2, e), \
            SP2State(st.i, st.xh, st.xl, e_hist)
    br = choose_branch(t1, t2, p.n_occ)
    xh, xl = map_gap(st.xh, br), map_gap(st.xl, br)
    delta = step_delta(p, xh - xl)
    taus = np.asarray(p.taus, dtype=np.float64)
    nu = norms(X)[1]
    budget = delta / 2.0 if p.variant == "hybrid" else delta
    if p.variant == "truncmul":
        bound, idx, tau = np.zeros(len(taus)), len(taus), 0.0
    else:
        skip_budget = p.tier_split * budget if p.precision else budget
        if p.bound == "tree":
            bound = cse_tree(X, X, taus, nu, nu)
        else:
            flat, ssum = cse_flat_sum(X, X, taus, nu, nu)
            bound = flat if p.bound == "flat" else ssum
        idx, tau = select(bound, taus, skip_budget)
    sidx, sigma, nlow = len(taus), 0.0, 0
    if p.precision:
        # the largest low-precision limit whose bound (skipped p, plus c p for
        # pairs evaluated in the low tier) stays below the product budget
        c_low = tier_constant(p.precision, X.b)
        if p.bound == "tree":
            bound2 = cse_tree(X, X, taus, nu, nu, mode=1, tau0=tau, c_low=c_low)
        else:
            f2, s2 = cse_flat_sum(X, X, taus, nu, nu, mode=1, tau0=tau, c_low=c_low)
            bound2 = f2 if p.bound == "flat" else s2
        sidx, sigma = select(bound2, taus, budget)
    C, K = spamm(X, X, tau, sym=True, nuA=nu, nuB=nu)
    if p.precision:
        nlow = low_tier_pairs(X, tau, sigma, nu, p.precision)
    Xh = combine(X, C, br)
    if p.variant == "spamm":
        Xt, ti = Xh.sorted(), None
    else:
        tb = delta / 2.0 if p.variant == "hybrid" else delta
        Xt, ti = truncate(Xh.sorted(), tb)
    log = StepLog(st.i, br, delta, bound, idx, tau, K.npairs, int(K.oi.shape[0]), ti, t1, t2, e, sidx, sigma, nlow)
    return Xt, Xh, log, SP2State(st.i + 1, xh, xl, e_hist)


def sp2_start(F: BSM, p: SP2Params):
    """X~_0 from F: Gerschgorin map (reading of 'a linear transformation'),
    then the first truncation with delta_0."""
    lmin, lmax = gerschgorin(F)
    X0 = x0(F, lmin, lmax)
    W = lmax - lmin
    xh = (lmax - p.homo) / W
    xl = (lmax - p.lumo) / W
    d0 = step_delta(p, xh - xl)
    if p.variant == "spamm":
        Xt, ti = X0, None
    else:
        Xt, ti = truncate(X0, d0)
    return Xt, X0, SP2State(1, xh, xl, []), (lmin, lmax, d0, ti)


def sp2(F: BSM, p: SP2Params, keep_tape: bool = False):
    """Full purification.  Returns (D~, logs, info)."""
    X, X0, st, info = sp2_start(F, p)
    logs = []
    tape = [X] if keep_tape else None
    while True:
        Xn, _, log, st = sp2_step(X, st, p)
        logs.append(log)
        if Xn is None:
            break
        X = Xn
        if keep_tape:
            tape.append(X)
    return X, logs, {"lmin": info[0], "lmax": info[1], "delta0": info[2], "tape": tape,
                     "converged": logs[-1].branch == -1 and st.i <= p.n_max}


# ---------------------------------------------------------------------------
# Reverse mode of the purification with frozen decisions (not in the paper).
#
# With the kept sets K_t, the truncation patterns S_t, the branches and the
# Gerschgorin bounds held fixed at their values in a forward run, the
# purification is a polynomial map F -> D~:
#   X~_0 = mask_{S_0}((lmax I - F) / (lmax - lmin)),
#   X~_t = mask_{S_t}(f_t(C_t(X~_{t-1}))),  C_t(X) = sum_{(i,k,j) in K_t} X_ik X_kj,
#   f_t(C) = C (x^2 branch) or 2 X~_{t-1} - C (2x - x^2 branch).
# Gradients are for symmetric perturbations: <Fbar, H> = dL[H] for every
# symmetric H, Fbar symmetric.
# ---------------------------------------------------------------------------

def _blocks(X: BSM) -> dict:
    """(r, c) -> row-major b x b block."""
    return {(int(X.brow[t]), int(X.bcol[t])): X.vals[t].T for t in range(X.nblk)}


def _from_blocks(X: BSM, blk: dict) -> BSM:
    """Values on X's pattern and block order from a (r, c) -> block dict
    (absent keys give zero blocks)."""
    b = X.b
    vals = np.zeros((X.nblk, b, b))
    for t in range(X.nblk):
        key = (int(X.brow[t]), int(X.bcol[t]))
        if key in blk:
            vals[t] = blk[key].T
    return BSM(X.n, b, X.brow.copy(), X.bcol.copy(), np.ascontiguousarray(vals))


def sym_part(D: BSM) -> BSM:
    """(D + D^T)/2 on D's pattern (which must be symmetric)."""
    d = _blocks(D)
    return _from_blocks(D, {(r, c): 0.5 * (v + d[(c, r)].T) for (r, c), v in d.items()})


def adjoint_step(X: BSM, G: BSM, tau: float, branch: int, nu=None) -> BSM:
    """Reverse of one frozen step X~' = mask_{S'}(f(C(X))) at X = X~_{t-1}.
    G is the (symmetric) gradient with respect to X~' on its pattern S', so
    mask_{S'} is already applied.  K = {(i,k,j): RN(nu(X_ik) nu(X_kj)) >= tau}
    is the leaf-level kept set of Algorithm 2 at X.  By the product rule,
      first factor   A_ik = sum_{j: (i,k,j) in K} G_ij X_kj^T,
      second factor  B_kj = sum_{i: (i,k,j) in K} X_ik^T G_ij,
    the gradient of <G, C(X)> is sym(A + B), and the step's gradient with
    respect to X, restricted to the pattern of X (outside it X~_{t-1} is an
    exact zero fixed by the previous truncation), is
      sym(A + B)            (x^2 branch),
      2 G - sym(A + B)      (2x - x^2 branch; G read as 0 outside S').
    Returns it on X's pattern and block order."""
    nu = norms(X)[1] if nu is None else nu
    K = kept(X, X, tau, False, nu, nu)       # all outputs (i, j), no symmetry shortcut
    xb, gb = _blocks(X), _blocks(G)
    acc = {}
    for o in range(K.oi.shape[0]):
        i, j = int(K.oi[o]), int(K.oj[o])
        if (i, j) not in gb:
            continue
        g = gb[(i, j)]
        for k in K.klist[K.kptr[o]:K.kptr[o + 1]]:
            k = int(k)
            a = g @ xb[(k, j)].T                 # first factor X_ik
            acc[(i, k)] = acc.get((i, k), 0.0) + a
            bb = xb[(i, k)].T @ g                # second factor X_kj
            acc[(k, j)] = acc.get((k, j), 0.0) + bb
    out = {}
    z = np.zeros((X.b, X.b))
    for (r, c) in xb:
        s = 0.5 * (acc.get((r, c), z) + acc.get((c, r), z).T)
        if branch == 1:
            s = 2.0 * gb.get((r, c), z) - s
        out[(r, c)] = s
    return _from_blocks(X, out)


def sp2_adjoint(F: BSM, tape: list, logs: list, lmin: float, lmax: float, Dbar: BSM) -> BSM:
    """Gradient of L with respect to F (on F's pattern and block order) from
    Dbar = dL/dD~ on the pattern of D~ = tape[-1], by the reverse of every
    frozen step (adjoint_step) and of X~_0 = mask_{S_0}((lmax I - F)/W):
    Fbar = -Xbar_0 / W on S_0, zero on blocks of F that the first truncation
    removed.  tape[t] = X~_t; logs[t-1] holds tau and the branch of step t."""
    G = sym_part(Dbar)
    for t in range(len(tape) - 1, 0, -1):
        lg = logs[t - 1]
        G = adjoint_step(tape[t - 1], G, lg.tau, lg.branch)
    W = lmax - lmin
    g0 = _blocks(G)
    return _from_blocks(F, {k: -v / W for k, v in g0.items()})


def _mask(X: BSM, S: BSM) -> BSM:
    """X restricted to the pattern of S, in S's block order (zeros where X
    has no block)."""
    return _from_blocks(S, _blocks(X))


def sp2_replay(F: BSM, tape: list, logs: list, lmin: float, lmax: float) -> BSM:
    """The frozen map F -> D~ of a recorded run: the kept set of step t is
    recomputed from tape[t-1] (the recorded iterate) and tau_t, the
    truncation keeps exactly the pattern of tape[t]."""
    X = _mask(x0(F, lmin, lmax), tape[0])
    for t in range(1, len(tape)):
        lg = logs[t - 1]
        Xr = tape[t - 1]
        nu = norms(Xr)[1]
        K = kept(Xr, Xr, lg.tau, True, nu, nu)
        V = block_products(X, X, K)
        off = K.oi != K.oj
        C = BSM(X.n, X.b, np.concatenate([K.oi, K.oj[off]]).astype(np.int32),
                np.concatenate([K.oj, K.oi[off]]).astype(np.int32),
                np.ascontiguousarray(np.concatenate([V, V[off].transpose(0, 2, 1)]))).sorted()
        X = _mask(combine(X, C, lg.branch), tape[t])
    return X
