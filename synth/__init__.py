"""Seeded synthetic workloads for SpAMM / SP2 purification.

This module only *produces inputs*: symmetric block-sparse Fock-like
matrices, weight matrices and candidate-threshold lists.  It contains none
of the method's arithmetic (no norms, bounds, products, truncation or
purification), so both the CPU oracle and the GPU library can consume its
output without sharing any computation.

The paper's workload (a converged Ergo density matrix of a water cluster,
n = 71253, Section "evaluation") is not available; the generators below
stand in for it with matrices that have the same qualitative structure:
exponential decay with distance, a spectral gap at half filling, and a
block-sparse quadtree pattern.

Random numbers come from one counter-based generator: the k-th output of
SplitMix64 (Steele, Lea and Flood, 2014) started from state 0,

    h(x) = mix((x + 1) * 0x9E3779B97F4A7C15 mod 2^64)
    mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
            z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31

with the counter x packing (seed, stream, index) as
seed << 44 | stream << 40 | index  (index < 2^40, stream < 16,
seed < 2^20).  U01 = (h >> 11) * 2^-53.

Block layout shared by every consumer: a matrix of order n with leaf size b
has nb = ceil(n / b) block rows; a present block (r, c) stores its b*b
values column-major, i.e. vals[k, col, row] = X[r*b + row, c*b + col];
rows/columns past n are zero padding.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, stream: int, index) -> np.ndarray:
    """Counter-based SplitMix64 output for (seed, stream, index) (uint64)."""
    if not (0 <= seed < (1 << 20) and 0 <= stream < 16):
        raise ValueError("seed must be < 2^20 and stream < 16")
    idx = np.asarray(index, dtype=np.uint64)
    if idx.size and int(idx.max()) >= (1 << 40):
        raise ValueError("index must be < 2^40")
    x = (np.uint64(seed) << np.uint64(44)) | (np.uint64(stream) << np.uint64(40)) | idx
    with np.errstate(over="ignore"):
        z = (x + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def u01(seed: int, stream: int, index) -> np.ndarray:
    """Uniform doubles in [0, 1) from the counter-based generator."""
    return (splitmix64(seed, stream, index) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class BlockMatrix:
    """Host-side block-sparse matrix in the shared layout (see module doc)."""

    n: int
    b: int
    brow: np.ndarray  # int32 [nblk]
    bcol: np.ndarray  # int32 [nblk]
    vals: np.ndarray  # float64 [nblk, b, b], vals[k, col, row]

    @property
    def nb(self) -> int:
        return (self.n + self.b - 1) // self.b

    @property
    def nblk(self) -> int:
        return int(self.brow.shape[0])

    def sorted(self) -> "BlockMatrix":
        """Same matrix with blocks in row-major (brow, bcol) order."""
        key = self.brow.astype(np.int64) * self.nb + self.bcol
        o = np.argsort(key, kind="stable")
        return BlockMatrix(self.n, self.b, self.brow[o].copy(), self.bcol[o].copy(),
                           np.ascontiguousarray(self.vals[o]))

    def to_dense(self) -> np.ndarray:
        nb, b = self.nb, self.b
        D = np.zeros((nb * b, nb * b))
        for k in range(self.nblk):
            r, c = int(self.brow[k]), int(self.bcol[k])
            D[r * b:(r + 1) * b, c * b:(c + 1) * b] = self.vals[k].T
        return D[: self.n, : self.n]

    @staticmethod
    def from_dense(D: np.ndarray, b: int, keep_zero_diag: bool = False) -> "BlockMatrix":
        """Blocks of D that hold any nonzero (plus, optionally, every diagonal block)."""
        n = D.shape[0]
        nb = (n + b - 1) // b
        P = np.zeros((nb * b, nb * b))
        P[:n, :n] = D
        T = P.reshape(nb, b, nb, b).transpose(0, 2, 3, 1)  # [r, c, col, row]
        present = np.any(T != 0.0, axis=(2, 3))
        if keep_zero_diag:
            present[np.arange(nb), np.arange(nb)] = True
        rr, cc = np.nonzero(present)
        return BlockMatrix(n, b, rr.astype(np.int32), cc.astype(np.int32),
                           np.ascontiguousarray(T[rr, cc]))


# ---------------------------------------------------------------------------
# Workload 1: one-dimensional two-band chain
# ---------------------------------------------------------------------------

def chain1d(n: int = 1024, seed: int = 1, b: int = 32, reach: int = 8) -> BlockMatrix:
    """F_ii = +1 (even i) / -1 (odd i); F_ij = 0.1 s_ij exp(-|i-j|/2) for
    0 < |i-j| <= reach, s_ij = +-1 from the top bit of h(seed, 0, i*n+j), i<j,
    mirrored."""
    F = np.zeros((n, n))
    i = np.arange(n)
    F[i, i] = np.where(i % 2 == 0, 1.0, -1.0)
    for d in range(1, reach + 1):
        a = np.arange(n - d)
        c = a + d
        h = splitmix64(seed, 0, (a * n + c).astype(np.uint64))
        s = np.where((h >> np.uint64(63)) == 0, 1.0, -1.0)
        v = 0.1 * s * math.exp(-d / 2.0)
        F[a, c] = v
        F[c, a] = v
    return BlockMatrix.from_dense(F, b)


# ---------------------------------------------------------------------------
# Workloads 2, 3, 5: three-dimensional random site system
# ---------------------------------------------------------------------------

RC2 = 2.0 * math.log(1e16)  # exp(-r^2/2) < 1e-16 beyond r^2 > RC2 (r ~ 8.58 A)


def _morton3(q: np.ndarray) -> np.ndarray:
    """30-bit Morton code of 10-bit integer coordinates q[:, 3]."""
    code = np.zeros(q.shape[0], dtype=np.int64)
    for bit in range(10):
        for d in range(3):
            code |= ((q[:, d] >> bit) & 1) << (3 * bit + d)
    return code


def sites3d(n: int, seed: int):
    """Site positions (Morton-sorted) and the box side for an order-n system."""
    nsites = (n + 2) // 3
    L = (nsites / 0.1) ** (1.0 / 3.0)
    pos = u01(seed, 0, np.arange(3 * nsites, dtype=np.uint64)).reshape(nsites, 3) * L
    q = np.minimum((pos / L * 1024.0).astype(np.int64), 1023)
    order = np.argsort(_morton3(q), kind="stable")
    return pos[order], L


def sys3d(n: int, seed: int, b: int = 64, chunk: int = 128) -> BlockMatrix:
    """Sites uniform in a cube at density 0.1 / A^3 (open boundaries), sorted
    by Morton code; basis function i sits on site floor(i/3).
    F_ii = +1 (even i) / -1 (odd i); for i < j,
    F_ij = -exp(-r_ij^2 / 2) * u_ij with u_ij = 0.5 + 0.5 U01(h(seed, 1, i*n+j)),
    structurally zero where r_ij^2 > RC2; mirrored."""
    pos, _ = sites3d(n, seed)
    nb = (n + b - 1) // b
    bpos = pos[np.arange(n) // 3]                      # (n, 3)
    pad = nb * b - n
    if pad:
        bpos = np.concatenate([bpos, np.full((pad, 3), np.nan)])
    bp = bpos.reshape(nb, b, 3)
    lo = np.nanmin(bp, axis=1)
    hi = np.nanmax(bp, axis=1)
    # candidate block pairs I <= J whose bounding boxes are within the cutoff
    gap = np.maximum(0.0, np.maximum(lo[:, None, :] - hi[None, :, :], lo[None, :, :] - hi[:, None, :]))
    d2 = np.sum(gap * gap, axis=2)
    I, J = np.nonzero(np.triu(d2 <= RC2))
    rows_out, cols_out, vals_out = [], [], []
    ar = np.arange(b)
    for s in range(0, I.shape[0], chunk):
        Ic, Jc = I[s:s + chunk], J[s:s + chunk]
        gi = Ic[:, None] * b + ar[None, :]             # (C, b) global rows
        gj = Jc[:, None] * b + ar[None, :]             # (C, b) global cols
        diff = bp[Ic][:, :, None, :] - bp[Jc][:, None, :, :]
        r2 = np.sum(diff * diff, axis=3)               # (C, b_row, b_col)
        valid = (gi[:, :, None] < gj[:, None, :]) & (gj[:, None, :] < n) & ~np.isnan(r2)
        valid &= r2 <= RC2
        ctr = (gi[:, :, None].astype(np.uint64) * np.uint64(n) + gj[:, None, :].astype(np.uint64))
        ctr = np.where(valid, ctr, np.uint64(0))
        u = 0.5 + 0.5 * u01(seed, 1, ctr)
        with np.errstate(invalid="ignore"):
            V = np.where(valid, -np.exp(-0.5 * np.where(valid, r2, 0.0)) * u, 0.0)  # V[c, row, col]
        diag = Ic == Jc
        if np.any(diag):
            k = np.nonzero(diag)[0]
            V[k] = V[k] + V[k].transpose(0, 2, 1)
            g = Ic[k][:, None] * b + ar[None, :]
            dv = np.where(g < n, np.where(g % 2 == 0, 1.0, -1.0), 0.0)
            V[k[:, None], ar[None, :], ar[None, :]] = dv
        keep = np.any(V != 0.0, axis=(1, 2)) | diag
        for c in np.nonzero(keep)[0]:
            Ib, Jb = int(Ic[c]), int(Jc[c])
            blk = V[c]                                  # blk[row, col]
            rows_out.append(Ib); cols_out.append(Jb); vals_out.append(blk.T)
            if Ib != Jb:
                rows_out.append(Jb); cols_out.append(Ib); vals_out.append(blk)
    M = BlockMatrix(n, b, np.array(rows_out, dtype=np.int32), np.array(cols_out, dtype=np.int32),
                    np.ascontiguousarray(np.array(vals_out).reshape(-1, b, b)))
    return M.sorted()


def band_w(n: int, b: int, bw: int = 64, seed: int = 55) -> BlockMatrix:
    """Symmetric banded W with W_ij ~ N(0,1) for |i-j| <= bw (Box-Muller on
    two streams of the counter generator, index i*n+j for i <= j)."""
    i_list, j_list = [], []
    for d in range(bw + 1):
        a = np.arange(n - d)
        i_list.append(a); j_list.append(a + d)
    ii = np.concatenate(i_list); jj = np.concatenate(j_list)
    ctr = (ii.astype(np.uint64) * np.uint64(n) + jj.astype(np.uint64))
    u1 = ((splitmix64(seed, 0, ctr) >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)
    u2 = u01(seed, 1, ctr)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    nb = (n + b - 1) // b
    W = {}
    for a, c, v in ((ii, jj, z), (jj, ii, z)):
        br, bc = a // b, c // b
        key = br.astype(np.int64) * nb + bc
        for kk in np.unique(key):
            W.setdefault(int(kk), np.zeros((b, b)))
        # scatter per block
        order = np.argsort(key, kind="stable")
        ks, rs, cs, vs = key[order], (a % b)[order], (c % b)[order], v[order]
        bounds = np.flatnonzero(np.diff(ks)) + 1
        for seg_k, seg_r, seg_c, seg_v in zip(np.split(ks, bounds), np.split(rs, bounds),
                                             np.split(cs, bounds), np.split(vs, bounds)):
            W[int(seg_k[0])][seg_c, seg_r] = seg_v      # stored [col, row]
    keys = np.array(sorted(W), dtype=np.int64)
    vals = np.stack([W[int(k)] for k in keys])
    return BlockMatrix(n, b, (keys // nb).astype(np.int32), (keys % nb).astype(np.int32), vals)


def batch_sizes(seed: int = 4, count: int = 64):
    """Sizes and seeds of the batched workload: n_s = floor(2048 * 16^U01(h(seed,0,s))),
    system seed 4000 + s."""
    u = u01(seed, 0, np.arange(count, dtype=np.uint64))
    ns = np.floor(2048.0 * 16.0 ** u).astype(np.int64)
    return [(int(ns[s]), 4000 + s) for s in range(count)]


def symmetric_direction(n: int, b: int, pattern: BlockMatrix, seed: int) -> BlockMatrix:
    """Random symmetric matrix with the block pattern of `pattern` (entries
    U(-1,1) from stream 2, index i*n+j for i <= j), used as a finite-difference
    direction."""
    nb = (n + b - 1) // b
    out = np.zeros_like(pattern.vals)
    ar = np.arange(b)
    for k in range(pattern.nblk):
        r, c = int(pattern.brow[k]), int(pattern.bcol[k])
        gi = r * b + ar[:, None]
        gj = c * b + ar[None, :]
        lo_ = np.minimum(gi, gj); hi_ = np.maximum(gi, gj)
        ctr = np.where((gi < n) & (gj < n), lo_ * n + hi_, 0).astype(np.uint64)
        v = 2.0 * u01(seed, 2, ctr) - 1.0
        v = np.where((gi < n) & (gj < n), v, 0.0)
        out[k] = v.T
    return BlockMatrix(n, b, pattern.brow.copy(), pattern.bcol.copy(), out)


# ---------------------------------------------------------------------------
# Candidate threshold lists (inputs to the sweep)
# ---------------------------------------------------------------------------

def tau_paper(N: int = 350) -> np.ndarray:
    """The paper's list: tau_1 = 1, tau_i = 0.9 tau_{i-1} (evaluation section)."""
    t = [1.0]
    for _ in range(N - 1):
        t.append(t[-1] * 0.9)
    return np.array(t)


def tau_log(N: int = 32, lo_exp: float = -16.0) -> np.ndarray:
    """N log-spaced candidates from 1 down to 10^lo_exp."""
    return np.array([10.0 ** (lo_exp * m / (N - 1)) for m in range(N)])
