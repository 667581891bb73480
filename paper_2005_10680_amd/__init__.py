"""Python binding of libspamm (SpAMM with error control, SP2 purification)
for AMD MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libspamm.so, called through its C ABI (include/spamm.h).  PyTorch
provides device memory (tensors) and the current HIP stream.  The library
must be built (``python paper_2005_10680_amd/build.py``); importing the
compute functions without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspamm.so")

SPAMM_OK = 0
SPAMM_EINVAL = -1
SPAMM_ECAPACITY = -2
SPAMM_EWORKSPACE = -3
SPAMM_EHIP = -4
SPAMM_ENOTSUP = -5
SPAMM_WNOCONV = 1
SPAMM_WTAUFALLBACK = 2

SYMMETRIC = 1
B_TRANSPOSED = 2
SYNC = 4
TIER_BF16 = 8
BOUND_FLAT = 16
BOUND_SUM = 32

VARIANTS = {"hybrid": 0, "spamm": 1, "truncmul": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
BOUNDS = {"tree": 0, "flat": 1, "sum": 2}


class SpammError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"spamm error {code}: {msg}")
        self.code = code


class spamm_bsm(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("b", ctypes.c_int32), ("nb", ctypes.c_int32), ("cap", ctypes.c_int64),
                ("nslot", ctypes.c_void_p), ("brow", ctypes.c_void_p), ("bcol", ctypes.c_void_p),
                ("map", ctypes.c_void_p), ("val", ctypes.c_void_p), ("norm", ctypes.c_void_p),
                ("sq", ctypes.c_void_p), ("sqlo", ctypes.c_void_p)]


class sp2_params(ctypes.Structure):
    _fields_ = [("n_occ", ctypes.c_int64), ("eps", ctypes.c_double), ("n_max", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("tau", ctypes.c_void_p), ("N", ctypes.c_int32),
                ("homo", ctypes.c_double), ("lumo", ctypes.c_double), ("delta_const", ctypes.c_double),
                ("e_tol", ctypes.c_double), ("keep_tape", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tier_split", ctypes.c_double), ("graph_steps", ctypes.c_int32), ("bound_kind", ctypes.c_int32)]


class sp2_iter_log(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int32), ("branch", ctypes.c_int32), ("idx", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("delta", ctypes.c_double), ("tau", ctypes.c_double), ("t1", ctypes.c_double),
                ("t2", ctypes.c_double), ("e", ctypes.c_double), ("npairs", ctypes.c_int64),
                ("nout", ctypes.c_int64), ("nslot_hat", ctypes.c_int64), ("nslot_kept", ctypes.c_int64),
                ("removed_units", ctypes.c_int64), ("removed_fro2", ctypes.c_double),
                ("ms_sweep", ctypes.c_float), ("ms_pairs", ctypes.c_float), ("ms_gemm", ctypes.c_float),
                ("ms_norms", ctypes.c_float), ("ms_trunc", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("npairs_low", ctypes.c_int64), ("sigma", ctypes.c_double), ("sidx", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libspamm.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2005_10680_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    B = ctypes.POINTER(spamm_bsm)
    u32 = ctypes.c_uint32
    L.spamm_build_norms.argtypes = [B, P]
    L.spamm_sweep_workspace_bytes.argtypes = [i32, i32]
    L.spamm_sweep_workspace_bytes.restype = sz
    L.spamm_sweep_tau.argtypes = [B, B, P, i32, P, d, i32, P, d, u32, P, P, P, P, sz, P]
    L.spamm_multiply_workspace_bytes.argtypes = [i32, i64]
    L.spamm_multiply_workspace_bytes.restype = sz
    L.spamm_multiply.argtypes = [B, B, P, u32, B, P, P, sz, P]
    L.spamm_truncate_workspace_bytes.argtypes = [i64]
    L.spamm_truncate_workspace_bytes.restype = sz
    L.spamm_truncate.argtypes = [B, d, u32, P, P, sz, P]
    L.spamm_truncate_noalloc_max_cap.argtypes = []
    L.spamm_truncate_noalloc_max_cap.restype = i64
    L.spamm_truncate_noalloc.argtypes = [B, d, u32, P, P]
    L.purify_sp2_workspace_bytes.argtypes = [i32, i32, i32, i64, i64, i32, i32]
    L.purify_sp2_workspace_bytes.restype = sz
    L.purify_sp2.argtypes = [B, ctypes.POINTER(sp2_params), B, ctypes.POINTER(sp2_iter_log),
                             ctypes.POINTER(i32), P, sz, P]
    L.purify_sp2_tape_view.argtypes = [P, i32, i32, i32, i64, i64, i32, i32, B]
    L.spamm_multiply_tiered_workspace_bytes.argtypes = [i32, i64, i64, i32, i64]
    L.spamm_multiply_tiered_workspace_bytes.restype = sz
    L.spamm_multiply_tiered.argtypes = [B, B, P, P, u32, B, P, P, sz, P]
    L.spamm_tier_constant.argtypes = [i32, i32]
    L.spamm_tier_constant.restype = d
    L.spamm_adjoint_step_workspace_bytes.argtypes = [i32, i64, i64]
    L.spamm_adjoint_step_workspace_bytes.restype = sz
    L.spamm_adjoint_step.argtypes = [B, B, d, i32, P, P, P, sz, P]
    L.purify_sp2_adjoint_workspace_bytes.argtypes = [i32, i32, i64, i64, i32]
    L.purify_sp2_adjoint_workspace_bytes.restype = sz
    L.purify_sp2_adjoint.argtypes = [B, ctypes.POINTER(sp2_params), B, i32, i32, B, ctypes.POINTER(sp2_iter_log),
                                     i32, P, P, P, sz, P]
    L.purify_sp2_batched_workspace_bytes.argtypes = [i32, B, ctypes.POINTER(sp2_params), P, P]
    L.purify_sp2_batched_workspace_bytes.restype = sz
    L.purify_sp2_batched.argtypes = [i32, B, ctypes.POINTER(sp2_params), B, P, ctypes.POINTER(sp2_iter_log), i32,
                                     P, P, P, sz, P]
    L.spamm_reblock_workspace_bytes.argtypes = [i32]
    L.spamm_reblock_workspace_bytes.restype = sz
    L.spamm_reblock.argtypes = [B, B, P, sz, P]
    L.spamm_set_gemm_schedule.argtypes = [i32, i32]
    L.spamm_get_gemm_schedule.argtypes = [i32]
    L.spamm_set_small_path.argtypes = [i32]
    L.spamm_get_small_path.argtypes = []
    L.purify_sp2_autotune_workspace_bytes.argtypes = [i64, i32, i32]
    L.purify_sp2_autotune_workspace_bytes.restype = sz
    L.purify_sp2_autotune.argtypes = [B, ctypes.POINTER(sp2_params), i32, P, P, P, P, sz, P]
    L.spamm_status_str.argtypes = [ctypes.c_int]
    L.spamm_status_str.restype = ctypes.c_char_p
    L.spamm_last_error.restype = ctypes.c_char_p
    L.spamm_version.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        raise SpammError(rc, lib().spamm_last_error().decode())
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class BlockSparse:
    """Block-sparse matrix in device memory (the spamm_bsm layout).

    Slots hold b*b doubles each, column-major inside a block; map[r*nb + c]
    is the slot of block (r, c) or -1; brow[slot] == -1 marks a hole."""

    def __init__(self, n: int, b: int, cap: int, device="cuda"):
        self.n, self.b = int(n), int(b)
        self.nb = (self.n + self.b - 1) // self.b
        self.cap = int(cap)
        dev = torch.device(device)
        i32 = torch.int32
        self.nslot = torch.zeros(1, dtype=i32, device=dev)
        self.brow = torch.full((self.cap,), -1, dtype=i32, device=dev)
        self.bcol = torch.full((self.cap,), -1, dtype=i32, device=dev)
        self.map = torch.full((self.nb * self.nb,), -1, dtype=i32, device=dev)
        self.val = torch.zeros(self.cap * self.b * self.b, dtype=torch.float64, device=dev)
        self.norm = torch.zeros(self.cap, dtype=torch.float64, device=dev)
        self.sq = torch.zeros(self.cap, dtype=torch.float64, device=dev)
        self.sqlo = torch.zeros(self.cap, dtype=torch.float64, device=dev)
        self._st = None

    @property
    def device(self):
        return self.val.device

    def struct(self) -> spamm_bsm:
        if self._st is None:
            self._st = spamm_bsm(self.n, self.b, self.nb, self.cap, self.nslot.data_ptr(), self.brow.data_ptr(),
                                 self.bcol.data_ptr(), self.map.data_ptr(), self.val.data_ptr(),
                                 self.norm.data_ptr(), self.sq.data_ptr(), self.sqlo.data_ptr())
        return self._st

    @classmethod
    def from_blocks(cls, n, b, brow, bcol, vals, cap=None, device="cuda") -> "BlockSparse":
        """From host arrays: brow/bcol [nblk], vals [nblk, b, b] with vals[k, col, row]."""
        brow = np.ascontiguousarray(brow, dtype=np.int32)
        bcol = np.ascontiguousarray(bcol, dtype=np.int32)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        nblk = brow.shape[0]
        cap = nblk if cap is None else max(int(cap), nblk)
        M = cls(n, b, max(cap, 1), device)
        nb = M.nb
        if nblk:
            M.brow[:nblk] = torch.from_numpy(brow).to(M.device)
            M.bcol[:nblk] = torch.from_numpy(bcol).to(M.device)
            M.val[: nblk * b * b] = torch.from_numpy(vals.reshape(-1)).to(M.device)
            mp = np.full(nb * nb, -1, dtype=np.int32)
            mp[brow.astype(np.int64) * nb + bcol] = np.arange(nblk, dtype=np.int32)
            M.map.copy_(torch.from_numpy(mp).to(M.device))
        M.nslot.fill_(nblk)
        return M

    @classmethod
    def from_host(cls, H, cap=None, device="cuda") -> "BlockSparse":
        """From any host object with n, b, brow, bcol, vals."""
        return cls.from_blocks(H.n, H.b, H.brow, H.bcol, H.vals, cap, device)

    @classmethod
    def wrap(cls, st: spamm_bsm, keepalive=None) -> "BlockSparse":
        """A view of device arrays described by a spamm_bsm (no copy)."""
        M = cls.__new__(cls)
        M.n, M.b, M.nb, M.cap = st.n, st.b, st.nb, st.cap
        M._st = st
        M._keep = keepalive
        dev = keepalive.device if keepalive is not None else torch.device("cuda")

        def view(ptr, count, dtype):
            return _DeviceView(ptr, count, dtype, dev)
        M.nslot = view(st.nslot, 1, torch.int32)
        M.brow = view(st.brow, st.cap, torch.int32)
        M.bcol = view(st.bcol, st.cap, torch.int32)
        M.map = view(st.map, st.nb * st.nb, torch.int32)
        M.val = view(st.val, st.cap * st.b * st.b, torch.float64)
        M.norm = view(st.norm, st.cap, torch.float64)
        M.sq = view(st.sq, st.cap, torch.float64)
        M.sqlo = view(st.sqlo, st.cap, torch.float64)
        return M

    def live(self):
        """Host copy of the live blocks, sorted row-major:
        (brow, bcol, vals[k, col, row], norm, sq, slots)."""
        torch.cuda.synchronize()
        ns = min(int(_host(self.nslot)[0]), self.cap)
        brow = _host(self.brow, ns)
        bcol = _host(self.bcol, ns)
        keep = np.nonzero(brow >= 0)[0]
        key = brow[keep].astype(np.int64) * self.nb + bcol[keep]
        o = keep[np.argsort(key, kind="stable")]
        b = self.b
        vals = _host(self.val, ns * b * b).reshape(ns, b, b)[o] if ns else np.zeros((0, b, b))
        return (brow[o].copy(), bcol[o].copy(), np.ascontiguousarray(vals), _host(self.norm, ns)[o].copy(),
                _host(self.sq, ns)[o].copy(), o)

    def block_map(self) -> np.ndarray:
        """Host copy of the block map: slot of block (r, c) at r * nb + c, or -1."""
        torch.cuda.synchronize()
        return _host(self.map)

    def blocks_at(self, rows, cols):
        """Host copies of the blocks (rows[t], cols[t]): (present[t], vals[t, col, row]),
        zeros where a block is absent; copies only those blocks."""
        b = self.b
        bmap = self.block_map()
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        slots = bmap[rows * self.nb + cols]
        out = np.zeros((rows.shape[0], b, b))
        for t, sl in enumerate(slots):
            if sl >= 0:
                out[t] = _host_range(self.val, int(sl) * b * b, b * b).reshape(b, b)
        return slots >= 0, out

    def to_host(self):
        """(n, b, brow, bcol, vals) of the live blocks as a plain record."""
        brow, bcol, vals, _, _, _ = self.live()
        return HostBlocks(self.n, self.b, brow, bcol, vals)


class _DeviceView:
    """Minimal typed view of raw device memory owned elsewhere."""

    def __init__(self, ptr, count, dtype, device):
        self.ptr, self.count, self.dtype, self.device = int(ptr), int(count), dtype, device

    def data_ptr(self):
        return self.ptr

    def numpy(self, count=None):
        npdt = {torch.int32: np.int32, torch.float64: np.float64}[self.dtype]
        out = np.empty(self.count if count is None else min(int(count), self.count), dtype=npdt)
        if out.size:
            hip_memcpy_d2h(out, self.ptr)
        return out


def _host(t, count=None) -> np.ndarray:
    """Host copy of t, or of its first count elements."""
    if isinstance(t, _DeviceView):
        return t.numpy(count)
    if count is not None:
        t = t[: int(count)]
    return t.detach().cpu().numpy()


def _host_range(t, start: int, count: int) -> np.ndarray:
    """Host copy of elements [start, start + count) of t."""
    if isinstance(t, _DeviceView):
        npdt = {torch.int32: np.int32, torch.float64: np.float64}[t.dtype]
        assert 0 <= start and start + count <= t.count
        out = np.empty(count, dtype=npdt)
        hip_memcpy_d2h(out, t.ptr + start * out.itemsize)
        return out
    return t[start:start + count].detach().cpu().numpy()


_hiprt = None


def hip_memcpy_d2h(out: np.ndarray, ptr: int):
    """Synchronous device-to-host copy (hipMemcpy) into a numpy array."""
    global _hiprt
    if _hiprt is None:
        _hiprt = ctypes.CDLL("libamdhip64.so")
        _hiprt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = _hiprt.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ptr), out.nbytes, 2)
    if rc != 0:
        raise SpammError(SPAMM_EHIP, f"hipMemcpy failed ({rc})")


@dataclass
class HostBlocks:
    n: int
    b: int
    brow: np.ndarray
    bcol: np.ndarray
    vals: np.ndarray


# ---------------------------------------------------------------------------
# the six operations
# ---------------------------------------------------------------------------

def build_norms(X: BlockSparse) -> None:
    """Exactly rounded block norms of every live slot (in place)."""
    _check(lib().spamm_build_norms(ctypes.byref(X.struct()), _stream()))


def sweep_tau(A: BlockSparse, B: BlockSparse, taus, budget, b_transposed=False, mode=0, tau0=None, c_low=0.0,
              sync=False, bound="tree", with_status=False):
    """Error bound of SpAMM(A, B, tau_k) for every candidate (Algorithm 3's
    recursive bound, or the leaf-level "flat" / "sum" bounds) and the
    selected candidate.  Returns device tensors (bound[N], idx[1], tau[1]),
    and with_status the call's status (with sync: SPAMM_WTAUFALLBACK when
    no candidate met the budget)."""
    kind_flag = {0: 0, 1: BOUND_FLAT, 2: BOUND_SUM}[BOUNDS[bound]]
    dev = A.device
    taus = torch.as_tensor(taus, dtype=torch.float64, device=dev).contiguous()
    N = int(taus.shape[0])
    bound = torch.empty(N, dtype=torch.float64, device=dev)
    idx = torch.empty(1, dtype=torch.int32, device=dev)
    tau = torch.empty(1, dtype=torch.float64, device=dev)
    ws = _ws(lib().spamm_sweep_workspace_bytes(A.nb, N), dev)
    bdev = budget if isinstance(budget, torch.Tensor) else None
    t0 = torch.as_tensor([tau0 if tau0 is not None else 0.0], dtype=torch.float64, device=dev)
    flags = (B_TRANSPOSED if b_transposed else 0) | (SYNC if sync else 0) | kind_flag
    rc = _check(lib().spamm_sweep_tau(ctypes.byref(A.struct()), ctypes.byref(B.struct()), _ptr(taus), N,
                                      _ptr(bdev) if bdev is not None else None,
                                      float(budget) if bdev is None else 0.0, int(mode), _ptr(t0), float(c_low),
                                      flags, _ptr(bound), _ptr(idx), _ptr(tau), _ptr(ws), ws.numel(), _stream()))
    return (bound, idx, tau, rc) if with_status else (bound, idx, tau)


def multiply(A: BlockSparse, B: BlockSparse, tau, symmetric=False, b_transposed=False, cap=None, max_pairs=None,
             out=None):
    """C~ = SpAMM(A, B, tau) (Algorithm 2).  Returns (C, kept[2] = pairs, outputs).
    out: an existing BlockSparse of the same n and leaf size to overwrite."""
    dev = A.device
    nb = A.nb
    if cap is None:
        cap = nb * nb
    if max_pairs is None:
        max_pairs = max(1, nb * nb * nb // (2 if symmetric else 1))
    C = out if out is not None else BlockSparse(A.n, A.b, cap, dev)
    tau_t = tau if isinstance(tau, torch.Tensor) else torch.tensor([float(tau)], dtype=torch.float64, device=dev)
    kept = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = _ws(lib().spamm_multiply_workspace_bytes(nb, 0) + 8 * int(max_pairs) + 1024, dev)
    flags = (SYMMETRIC if symmetric else 0) | (B_TRANSPOSED if b_transposed else 0)
    _check(lib().spamm_multiply(ctypes.byref(A.struct()), ctypes.byref(B.struct()), _ptr(tau_t), flags,
                                ctypes.byref(C.struct()), _ptr(kept), _ptr(ws), ws.numel(), _stream()))
    return C, kept


def multiply_tiered(A: BlockSparse, B: BlockSparse, tau, sigma, symmetric=False, b_transposed=False, cap=None,
                    max_pairs=None, tier="fp32"):
    """SpAMM with a low-precision tier ("fp32" or "bf16x3") for pairs with
    tau <= p < sigma.  Returns (C, kept[3] = pairs, outputs, low-tier pairs)."""
    dev = A.device
    nb = A.nb
    if cap is None:
        cap = nb * nb
    if max_pairs is None:
        max_pairs = max(1, nb * nb * nb // (2 if symmetric else 1))
    C = BlockSparse(A.n, A.b, cap, dev)
    tau_t = torch.tensor([float(tau)], dtype=torch.float64, device=dev)
    sig_t = torch.tensor([float(sigma)], dtype=torch.float64, device=dev)
    kept = torch.zeros(3, dtype=torch.int64, device=dev)
    base = lib().spamm_multiply_tiered_workspace_bytes(nb, A.cap, B.cap, A.b, 0)
    ws = _ws(base + 8 * int(max_pairs) + 1024, dev)
    flags = (SYMMETRIC if symmetric else 0) | (B_TRANSPOSED if b_transposed else 0) | \
        ({"fp32": 0, "bf16x3": TIER_BF16}[tier])
    _check(lib().spamm_multiply_tiered(ctypes.byref(A.struct()), ctypes.byref(B.struct()), _ptr(tau_t), _ptr(sig_t),
                                       flags, ctypes.byref(C.struct()), _ptr(kept), _ptr(ws), ws.numel(), _stream()))
    return C, kept


def tier_constant(precision: int, b: int) -> float:
    """Per-pair rounding factor c_t of a precision tier (1 = FP32)."""
    return float(lib().spamm_tier_constant(int(precision), int(b)))


def truncate(X: BlockSparse, delta: float, sync=False):
    """Remove symmetric units with ||E||_F < delta (in place).  Returns
    removed[2] = (units, bound of the removed squared norm)."""
    dev = X.device
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    ws = _ws(lib().spamm_truncate_workspace_bytes(X.cap), dev)
    _check(lib().spamm_truncate(ctypes.byref(X.struct()), float(delta), SYNC if sync else 0, _ptr(out), _ptr(ws),
                                ws.numel(), _stream()))
    return out


def truncate_noalloc(X: BlockSparse, delta: float, sync=False):
    """truncate() through the allocation-free entry point (the library's
    fixed scratch array instead of a workspace; X.cap <= 2^20)."""
    out = torch.zeros(2, dtype=torch.float64, device=X.device)
    _check(lib().spamm_truncate_noalloc(ctypes.byref(X.struct()), float(delta), SYNC if sync else 0, _ptr(out),
                                        _stream()))
    return out


@dataclass
class PurifyResult:
    D: BlockSparse
    logs: list
    status: int
    ws: torch.Tensor
    tape_args: tuple | None
    raw_logs: object = None
    nlog: int = 0
    tape_every: int = 0
    params: object = None     # the sp2_params of the run (kept with its tau tensor)
    taus: object = None

    def tape(self, step: int) -> BlockSparse:
        """X~_step of a run with keep_tape (a view into the workspace)."""
        if self.tape_args is None:
            raise ValueError("purify was run without keep_tape")
        st = spamm_bsm()
        _check(lib().purify_sp2_tape_view(_ptr(self.ws), *self.tape_args, int(step), ctypes.byref(st)))
        return BlockSparse.wrap(st, keepalive=self.ws)


def purify(F: BlockSparse, n_occ: int, eps: float, taus, homo=float("nan"), lumo=float("nan"),
           variant="hybrid", n_max=60, delta_const=float("nan"), e_tol=0.0, cap=None, max_pairs=None,
           keep_tape=False, precision="fp64", tier_split=0.5, graph_steps=0, bound="tree") -> PurifyResult:
    """SP2 purification with SpAMM and error control (Algorithms 1, 4, 5).
    graph_steps > 0: the step runs as a replayed HIP graph with its
    decisions taken on the device, the host polling every graph_steps
    iterations (keep_tape must be off; phase timings are 0)."""
    dev = F.device
    nb, b = F.nb, F.b
    taus = torch.as_tensor(taus, dtype=torch.float64, device=dev).contiguous()
    N = int(taus.shape[0])
    if cap is None:
        cap = nb * nb
    if max_pairs is None:
        max_pairs = max(1, nb * nb * (nb + 1) // 2)
    every = int(keep_tape)
    tape_steps = n_max if every == 1 else (n_max // every if every > 1 else 0)
    prec = PRECISIONS[precision]
    base = lib().purify_sp2_workspace_bytes(nb, b, N, int(cap), 0, tape_steps, prec)
    ws = _ws(base + 8 * int(max_pairs) + 1024, dev)
    mp = (ws.numel() - base - 512) // 8   # the pair capacity the library derives
    D = BlockSparse(F.n, b, cap, dev)
    p = sp2_params(int(n_occ), float(eps), int(n_max), VARIANTS[variant], taus.data_ptr(), N, float(homo),
                   float(lumo), float(delta_const), float(e_tol), every, prec, float(tier_split),
                   int(graph_steps), BOUNDS[bound])
    logs = (sp2_iter_log * (n_max + 2))()
    nlog = ctypes.c_int32(0)
    rc = lib().purify_sp2(ctypes.byref(F.struct()), ctypes.byref(p), ctypes.byref(D.struct()), logs,
                          ctypes.byref(nlog), _ptr(ws), ws.numel(), _stream())
    _check(rc)
    out = [{k: getattr(logs[i], k) for k, _ in sp2_iter_log._fields_} for i in range(nlog.value)]
    targs = (nb, b, N, int(cap), int(mp), tape_steps) if every else None
    return PurifyResult(D, out, rc, ws, targs, logs, nlog.value, every, p, taus)


@dataclass
class BatchResult:
    D: list        # BlockSparse per system
    logs: list     # per system: list of record dicts
    status: list   # per system
    rc: int        # worst status


def purify_batched(Fs, n_occ, eps, taus, homo, lumo, variant="hybrid", n_max=60, delta_const=float("nan"),
                   e_tol=0.0, caps=None, max_pairs=None, precision="fp64", tier_split=0.5, graph_steps=8,
                   raise_on_error=True, bound="tree") -> BatchResult:
    """Purify independent systems together (purify_sp2_batched): per step one
    persistent product launch for all systems of a leaf size and tier.
    Per-system arguments (n_occ, homo, lumo, taus, variant, precision,
    caps, max_pairs) are lists or one value for all."""
    ns = len(Fs)

    def per(v):
        return list(v) if isinstance(v, (list, tuple)) else [v] * ns
    n_occ, homo, lumo, variant, precision = per(n_occ), per(homo), per(lumo), per(variant), per(precision)
    bound = per(bound)
    taus_l = taus if isinstance(taus, (list, tuple)) else [taus] * ns
    dev = Fs[0].device
    tt = [torch.as_tensor(t, dtype=torch.float64, device=dev).contiguous() for t in taus_l]
    caps = per(caps) if caps is not None else [F.nb * F.nb for F in Fs]
    mps = per(max_pairs) if max_pairs is not None else [max(1, F.nb * F.nb * (F.nb + 1) // 2) for F in Fs]
    Fa = (spamm_bsm * ns)(*[F.struct() for F in Fs])
    Ds = [BlockSparse(F.n, F.b, int(cp), dev) for F, cp in zip(Fs, caps)]
    Da = (spamm_bsm * ns)(*[D.struct() for D in Ds])
    pa = (sp2_params * ns)()
    for q in range(ns):
        pa[q] = sp2_params(int(n_occ[q]), float(eps), int(n_max), VARIANTS[variant[q]], tt[q].data_ptr(),
                           int(tt[q].shape[0]), float(homo[q]), float(lumo[q]), float(delta_const), float(e_tol), 0,
                           PRECISIONS[precision[q]], float(tier_split), int(graph_steps), BOUNDS[bound[q]])
    capa = (ctypes.c_int64 * ns)(*[int(c) for c in caps])
    mpa = (ctypes.c_int64 * ns)(*[int(m) for m in mps])
    need = lib().purify_sp2_batched_workspace_bytes(ns, Fa, pa, capa, mpa)
    if need == 0:
        raise ValueError("bad batch arguments")
    ws = _ws(need, dev)
    stride = n_max + 2
    logs = (sp2_iter_log * (ns * stride))()
    nlog = (ctypes.c_int32 * ns)()
    st = (ctypes.c_int32 * ns)()
    rc = lib().purify_sp2_batched(ns, Fa, pa, Da, mpa, logs, stride, nlog, st, _ptr(ws), ws.numel(), _stream())
    if rc < 0 and raise_on_error:
        _check(rc)
    out = [[{k: getattr(logs[q * stride + i], k) for k, _ in sp2_iter_log._fields_} for i in range(nlog[q])]
           for q in range(ns)]
    return BatchResult(Ds, out, [int(x) for x in st], int(rc))


def reblock(X: BlockSparse, b: int, cap=None) -> BlockSparse:
    """The same matrix on leaf size b (spamm_reblock), norms included."""
    nb = (X.n + b - 1) // b
    Y = BlockSparse(X.n, b, int(cap) if cap is not None else nb * nb, X.device)
    ws = _ws(lib().spamm_reblock_workspace_bytes(nb), X.device)
    _check(lib().spamm_reblock(ctypes.byref(X.struct()), ctypes.byref(Y.struct()), _ptr(ws), ws.numel(), _stream()))
    return Y


def set_gemm_schedule(b: int, workgroups_per_cu: int) -> None:
    _check(lib().spamm_set_gemm_schedule(int(b), int(workgroups_per_cu)))


def get_gemm_schedule(b: int) -> int:
    return _check(lib().spamm_get_gemm_schedule(int(b)))


def set_small_path(on: bool) -> None:
    _check(lib().spamm_set_small_path(1 if on else 0))


def get_small_path() -> bool:
    return bool(_check(lib().spamm_get_small_path()))


def autotune(F: BlockSparse, n_occ: int, eps: float, taus, homo=float("nan"), lumo=float("nan"), variant="hybrid",
             n_max=60, delta_const=float("nan"), precision="fp64", tier_split=0.5, trial_steps=6):
    """Leaf size and product schedule for this input (purify_sp2_autotune):
    returns (best leaf size, workgroups per CU, {leaf: mean ms per step}).
    The schedule is installed process-wide."""
    dev = F.device
    taus = torch.as_tensor(taus, dtype=torch.float64, device=dev).contiguous()
    prec = PRECISIONS[precision]
    p = sp2_params(int(n_occ), float(eps), int(n_max), VARIANTS[variant], taus.data_ptr(), int(taus.shape[0]),
                   float(homo), float(lumo), float(delta_const), 0.0, 0, prec, float(tier_split), 0, 0)
    ws = _ws(lib().purify_sp2_autotune_workspace_bytes(F.n, int(taus.shape[0]), prec), dev)
    bb = ctypes.c_int32(0)
    pc = ctypes.c_int32(0)
    ms = (ctypes.c_float * 3)()
    _check(lib().purify_sp2_autotune(ctypes.byref(F.struct()), ctypes.byref(p), int(trial_steps), ctypes.byref(bb),
                                     ctypes.byref(pc), ms, _ptr(ws), ws.numel(), _stream()))
    del ws
    return int(bb.value), int(pc.value), {b: float(ms[q]) for q, b in enumerate((32, 64, 128)) if ms[q] >= 0}


def adjoint_step(X: BlockSparse, G: BlockSparse, tau: float, branch: int, max_pairs=None):
    """Reverse of one frozen purification step (spamm_adjoint_step): the
    gradient with respect to X on X's slot layout, from the symmetric
    gradient G on the pattern of the step's output.  Returns (xbar values
    [X.cap*b*b], device int64[2] = (output blocks, block pairs))."""
    nb, b = X.nb, X.b
    if max_pairs is None:
        max_pairs = max(1, nb * nb * (nb + 1))
    base = lib().spamm_adjoint_step_workspace_bytes(nb, X.cap, 0)
    ws = _ws(base + 8 * int(max_pairs) + 1024, X.device)
    xbar = torch.zeros(X.cap * b * b, dtype=torch.float64, device=X.device)
    counts = torch.zeros(2, dtype=torch.int64, device=X.device)
    _check(lib().spamm_adjoint_step(ctypes.byref(X.struct()), ctypes.byref(G.struct()), float(tau), int(branch),
                                    xbar.data_ptr(), counts.data_ptr(), _ptr(ws), ws.numel(), _stream()))
    return xbar, counts


def with_values(M: BlockSparse, val: torch.Tensor) -> BlockSparse:
    """M's pattern arrays with another value array (no copy)."""
    st = M.struct()
    st2 = spamm_bsm(st.n, st.b, st.nb, st.cap, st.nslot, st.brow, st.bcol, st.map, val.data_ptr(), st.norm, st.sq,
                    st.sqlo)
    return BlockSparse.wrap(st2, keepalive=val)


def purify_adjoint(res: PurifyResult, F: BlockSparse, dbar: torch.Tensor, max_pairs=None) -> torch.Tensor:
    """dL/dF (values in F's slot layout) from dbar = dL/dD~ (values in the
    slot layout of res.D) through the recorded run res (purify with
    keep_tape = 1, or k > 1 for checkpoints every k iterates), decisions
    held fixed (purify_sp2_adjoint)."""
    if res.tape_args is None:
        raise ValueError("purify was run without keep_tape")
    nb, b = F.nb, F.b
    every = res.tape_every
    steps = res.nlog - 1
    ntape = res.nlog if every == 1 else steps // every + 1
    tape = (spamm_bsm * ntape)()
    for t in range(ntape):
        _check(lib().purify_sp2_tape_view(_ptr(res.ws), *res.tape_args, t, ctypes.byref(tape[t])))
    cap = res.tape_args[3]
    if max_pairs is None:
        max_pairs = max(1, nb * nb * (nb + 1))
    base = lib().purify_sp2_adjoint_workspace_bytes(nb, b, cap, 0, every)
    ws = _ws(base + (16 if every > 1 else 8) * int(max_pairs) + 1024, F.device)
    dbar = dbar.to(torch.float64).contiguous()
    if dbar.numel() < cap * b * b:
        raise ValueError("dbar must hold the slots of D")
    fbar = torch.zeros(F.cap * b * b, dtype=torch.float64, device=F.device)
    _check(lib().purify_sp2_adjoint(ctypes.byref(F.struct()), ctypes.byref(res.params), tape, ntape, every,
                                    ctypes.byref(res.D.struct()), res.raw_logs, res.nlog, dbar.data_ptr(),
                                    fbar.data_ptr(), _ptr(ws), ws.numel(), _stream()))
    return fbar


class _Purify(torch.autograd.Function):
    """F values -> D~ values; backward through purify_sp2_adjoint."""

    @staticmethod
    def forward(ctx, fval, F, kw, holder):
        Fv = with_values(F, fval.detach().contiguous())
        kw = dict(kw)
        every = int(kw.pop("checkpoint_every", 1))
        res = purify(Fv, keep_tape=every, **kw)
        ctx.res, ctx.F = res, Fv
        holder["res"] = res
        return res.D.val

    @staticmethod
    def backward(ctx, dval):
        return purify_adjoint(ctx.res, ctx.F, dval), None, None, None


def purify_autograd(F: BlockSparse, fval: torch.Tensor, n_occ: int, eps: float, taus, **kw):
    """Differentiable purification: returns (D~ values, PurifyResult); the
    values are in the slot layout of result.D.  Gradients flow to fval (F's
    value array, F's slot layout) for symmetric perturbations, with the
    run's decisions (kept sets, truncation patterns, branches, Gerschgorin
    bounds) held fixed.  checkpoint_every = k > 1 keeps every k-th iterate
    and recomputes the others in the backward pass (FP64 runs)."""
    holder = {}
    dval = _Purify.apply(fval, F, dict(kw, n_occ=n_occ, eps=eps, taus=taus), holder)
    return dval, holder["res"]


def version() -> int:
    return int(lib().spamm_version())
