"""Benchmark: SP2 hybrid purification with error-controlled SpAMM on one
MI355X.

A step is one whole purification (every stage of the hot path: starting
matrix, block norms, traces and branch choice, the threshold sweep, kept
pairs, leaf products, combine and truncation, until the stop rule) of the
synthetic 3D system n = 16384, leaf 64, 32 candidate thresholds, eps = 1e-6,
with the input resident in HBM.  value = executed kept-pair flops (2 b^3 per
pair, i <= j outputs) over the whole timed purification.

Besides the timed steps the line carries: ||D - D~||_F of every
purification against the exact projector from a dense eigensolver (outside
the timed regions); the same purification as a replayed graph, selecting
with B_flat, and with the FP32 and split-BF16 leaf-product tiers; the
paper's three purification variants (Algorithms 5, 4, 1); the paper's
multiplication experiment on the converged D~ (SpAMM at the swept threshold,
exact product plus truncation, and SpAMM plus truncation at half the budget
each, delta = 1e-6, 1e-8, 1e-10); the small chain; the n = 65536 system in
FP64 and both tiers against a reference run; the reverse mode at n = 32768
with a finite-difference check; the 64-system batched workload in FP64 and
FP32 against the same systems run one after another; the oracle timed on a
sample of the workload and on the whole chain purification (cpu_baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-verify]
                    [--no-adjoint] [--batch N] [--no-big] [--no-protocol] [--no-mixed]
                    [--no-variants]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpAMM kept-block TFLOP/s; SP2 time to ||D−D̃||_F<1e-6, mixed vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_spectrum(name):
    path = os.path.join(ROOT, "tests", "golden", "spectra.json")
    with open(path) as f:
        return json.load(f)[name]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-verify", action="store_true",
                    help="skip the dense-eigensolver check of ||D - D~||_F (on by default, outside the timed region)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision purification")
    ap.add_argument("--graph", type=int, default=8,
                    help="also time the graph-captured loop, polling every K iterations (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the reverse mode on the n = 32768 system with a banded W (checkpointed tape)")
    ap.add_argument("--batch", type=int, default=64,
                    help="systems of the batched workload to time (the first N of the 64 systems, sizes "
                         "log-uniform in [2048, 32768], seed 4, leaf sizes by the autotuner; 0: skip)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the three purification variants (Algorithms 5, 4 and 1) on the main workload")
    ap.add_argument("--no-protocol", action="store_true",
                    help="skip the paper's multiplication experiment on the converged D~ "
                         "(delta = 1e-6, 1e-8, 1e-10)")
    ap.add_argument("--no-big", action="store_true",
                    help="skip the n = 65536 system (FP64 and both precision tiers against a reference run)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import synth
    batch_mats = None
    if args.batch > 0:
        # host-side generation first, before this process touches the GPU
        batch_mats = generate_batch(args.batch, synth)
    import torch
    import paper_2005_10680_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, b = args.n, args.leaf
    name = f"sys3d_n{n}_s{args.seed}_b{b}"
    spec = load_spectrum(name)
    n_occ = n // 2
    Fh = synth.sys3d(n, args.seed, b)
    taus = synth.tau_log(32)
    F = P.BlockSparse.from_host(Fh)
    nb = F.nb
    cap = nb * nb
    max_pairs = nb * nb * (nb + 1) // 2
    eps = 1e-6

    def run_once(precision="fp64", graph_steps=0, keep_tape=False, cap_=None, bound="tree", variant="hybrid",
                 taus_=None):
        return P.purify(F, n_occ, eps, taus if taus_ is None else taus_, homo=spec["homo"], lumo=spec["lumo"],
                        cap=cap_ or cap,
                        max_pairs=max_pairs, precision=precision, graph_steps=graph_steps, keep_tape=keep_tape,
                        bound=bound, variant=variant)

    log(f"input ready: n={n} leaf={b} blocks={Fh.nblk}")
    for w in range(args.warmup):
        run_once()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    times, flops, gemm_ms, gemm_flops, logs_all = [], 0.0, 0.0, 0.0, []
    res = None
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = run_once()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        steps = [l for l in res.logs if l["branch"] >= 0]
        log(f"step {len(times)}/{args.steps}: {times[-1]:.3f} s, {len(steps)} iterations")
        f = sum(l["npairs"] for l in steps) * 2.0 * b ** 3
        flops += f
        gemm_ms += sum(l["ms_gemm"] for l in steps)
        gemm_flops += f
        logs_all.append(res.logs)
    total_s = sum(times)
    value = flops / total_s / 1e12

    # the exact projector D = theta(mu - F) from a dense eigensolver (outside
    # every timed region), for ||D - D~||_F of each purification below
    dref = None
    if not args.no_verify:
        t0 = time.perf_counter()
        Fd = torch.from_numpy(Fh.to_dense()).to(dev)
        _, U = torch.linalg.eigh(Fd)
        del Fd
        Uo = U[:, :n_occ].contiguous()
        del U
        dref = Uo @ Uo.T
        del Uo
        torch.cuda.synchronize()
        log(f"dense reference projector in {time.perf_counter() - t0:.1f} s")

    def verify_err(r):
        """||D - D~||_F of a purification result (None without the reference)."""
        if dref is None:
            return None
        Dh = r.D.to_host()
        Dd = torch.zeros((n, n), dtype=torch.float64, device=dev)
        for k in range(Dh.brow.shape[0]):
            rr, cc = int(Dh.brow[k]), int(Dh.bcol[k])
            blk = torch.from_numpy(np.ascontiguousarray(Dh.vals[k].T)).to(dev)
            nr, nc = min(b, n - rr * b), min(b, n - cc * b)
            Dd[rr * b:rr * b + nr, cc * b:cc * b + nc] = blk[:nr, :nc]
        e = float(torch.linalg.norm(Dd - dref).item())
        del Dd
        return e
    steps = [l for l in res.logs if l["branch"] >= 0]
    ngemm = len(steps) * args.steps
    avg_gemm_ms = gemm_ms / ngemm
    achieved = (gemm_flops / ngemm) / (avg_gemm_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total_s / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sp2_hybrid_sys3d_n{n}_leaf{b}_tau32_eps1e-6", "n": n, "leaf": b,
                   "candidates": 32, "eps": eps, "variant": "hybrid", "n_occ": n_occ, "seed": args.seed},
        "sp2_time_s": round(float(np.median(times)), 4),
        "verify_fro_err": verify_err(res),
        "iterations": len(steps),
        "kept_pairs_per_run": int(sum(l["npairs"] for l in steps)),
        "phase_ms_per_run": {k: round(sum(l[k] for l in steps), 3)
                             for k in ("ms_sweep", "ms_pairs", "ms_gemm", "ms_norms", "ms_trunc", "ms_total")},
        # the purification takes its block norms from the product epilogue;
        # the stand-alone norms pass (spamm_build_norms, 8 b^2 bytes read per
        # block) over the converged D~, for its HBM rate
        "hbm_norms": norms_rate(res.D, b),
        "roofline": {"kernel": f"k_gemm_ring<{b},0>", "bound": "mfma", "achieved": round(achieved, 3),
                     "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(n, b, args.seed),
                     "avg_launch_ms": round(avg_gemm_ms, 4),
                     "flops_per_launch": gemm_flops / ngemm},
        "product_kernel": product_kernel_stats("fp64", b, int(sum(l["npairs"] for l in steps)), 0,
                                               sum(l["ms_gemm"] for l in steps), len(steps)),
    }

    # the same purification as a replayed graph with decisions on the device
    if args.graph > 0:
        run_once(graph_steps=args.graph)
        gtimes = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rg = run_once(graph_steps=args.graph)
            torch.cuda.synchronize()
            gtimes.append(time.perf_counter() - t0)
        gsteps = [l for l in rg.logs if l["branch"] >= 0]
        same = sum(l["npairs"] for l in gsteps) == sum(l["npairs"] for l in steps) and len(gsteps) == len(steps)
        log(f"graph loop: {float(np.median(gtimes)):.3f} s, {len(gsteps)} iterations")
        out["graph_loop"] = {"poll_every": args.graph, "sp2_time_s": round(float(np.median(gtimes)), 4),
                             "kept_TFLOP_per_s": round(flops / args.steps / float(np.median(gtimes)) / 1e12, 4),
                             "speedup_vs_host_loop": round(float(np.median(times)) / float(np.median(gtimes)), 4),
                             "same_decisions": bool(same)}

    # the same purification selecting tau (and sigma) with the leaf-level bound B_flat
    if not args.no_mixed:
        for prec, key in (("fp64", "bound_flat"), ("bf16x3", "bound_flat_bf16x3")):
            run_once(prec, bound="flat")
            ftimes = []
            for _ in range(args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rf = run_once(prec, bound="flat")
                torch.cuda.synchronize()
                ftimes.append(time.perf_counter() - t0)
            fsteps = [l for l in rf.logs if l["branch"] >= 0]
            fpairs = sum(l["npairs"] for l in fsteps)
            flow = sum(l["npairs_low"] for l in fsteps)
            log(f"B_flat selection ({prec}): {float(np.median(ftimes)):.3f} s, {len(fsteps)} iterations, "
                f"kept pairs {fpairs} ({flow} low tier)")
            out[key] = {"precision": prec, "sp2_time_s": round(float(np.median(ftimes)), 4),
                        "iterations": len(fsteps), "kept_pairs_per_run": int(fpairs),
                        "low_tier_pairs_per_run": int(flow),
                        "kept_pairs_vs_tree_fp64": round(fpairs / max(1, sum(l["npairs"] for l in steps)), 4),
                        "speedup_vs_fp64_tree": round(float(np.median(times)) / float(np.median(ftimes)), 4),
                        "mean_tau_ratio_vs_tree_fp64": round(float(np.exp(np.mean(
                            [np.log(a["tau"] / b["tau"]) for a, b in zip(fsteps, steps)
                             if a["tau"] > 0 and b["tau"] > 0]))), 3),
                        "verify_fro_err": verify_err(rf)}
            del rf

    # mixed precision (FP32 and split-BF16 leaf-product tiers) on the same workload
    if not args.no_mixed:
        for tier, key in (("fp32", "mixed"), ("bf16x3", "mixed_bf16x3")):
            run_once(tier)
            mtimes = []
            for _ in range(args.steps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rm = run_once(tier)
                torch.cuda.synchronize()
                mtimes.append(time.perf_counter() - t0)
            msteps = [l for l in rm.logs if l["branch"] >= 0]
            mpairs = sum(l["npairs"] for l in msteps)
            mlow = sum(l["npairs_low"] for l in msteps)
            log(f"{tier} tier: {float(np.median(mtimes)):.3f} s, {len(msteps)} iterations, "
                f"low-tier share {mlow / max(mpairs, 1):.3f}")
            out[key] = {"precision": f"{tier} tier", "sp2_time_s": round(float(np.median(mtimes)), 4),
                        "iterations": len(msteps), "kept_pairs_per_run": int(mpairs),
                        "low_tier_pairs_per_run": int(mlow),
                        "kept_TFLOP_per_s": round(mpairs * 2.0 * b ** 3 / float(np.median(mtimes)) / 1e12, 4),
                        "speedup_vs_fp64": round(float(np.median(times)) / float(np.median(mtimes)), 4),
                        "phase_ms_per_run": {k: round(sum(l[k] for l in msteps), 3)
                                             for k in ("ms_sweep", "ms_pairs", "ms_gemm", "ms_norms", "ms_trunc")},
                        "product_kernel": product_kernel_stats(tier, b, mpairs, mlow,
                                                               sum(l["ms_gemm"] for l in msteps), len(msteps)),
                        "verify_fro_err": verify_err(rm)}
            del rm

    # candidate lists: length and first candidate (the paper's closing
    # discussion names the threshold vector as a tuning knob)
    if not args.no_variants:
        out["candidate_lists"] = candidate_list_leg(run_once, torch, args.steps, b, synth)

    # the paper's three purification variants on the same workload:
    # Algorithm 5 (hybrid), 4 (SpAMM only) and 1 (exact product + truncation)
    if not args.no_variants:
        out["variants"] = variants_leg(run_once, torch, args.steps, b, eps, verify_err)

    if dref is not None:
        errs = [out["verify_fro_err"]] + [out[k]["verify_fro_err"] for k in
                                          ("bound_flat", "bound_flat_bf16x3", "mixed", "mixed_bf16x3") if k in out]
        log("verified: " + ", ".join(f"{e:.3e}" for e in errs))
        del dref
        dref = None
        torch.cuda.empty_cache()

    if args.copy_mb:
        src = torch.ones(args.copy_mb * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"plain copy of {args.copy_mb} MiB done")
        del src, dst

    if not args.no_protocol:
        out["protocol"] = protocol_leg(P, torch, res.D, taus)
        out["chain1024"] = chain_leg(P, torch, synth)

    if not args.no_big:
        keep = res
        out["big"] = big_leg(P, torch, synth)
        res = keep
        torch.cuda.empty_cache()

    # reverse mode at n = 32768 with a banded W (checkpointed tape)
    if not args.no_adjoint:
        torch.cuda.empty_cache()
        out["adjoint"] = adjoint_leg(dev, P, synth, torch)
        torch.cuda.empty_cache()

    if args.batch > 0:
        out["batched"] = batch_leg(args, dev, P, synth, batch_mats)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("timing the oracle on a sample (cpu baseline)")
        out["cpu_baseline"] = cpu_baseline(res, Fh, taus, b, args.cpu_seconds)
        out["cpu_baseline_chain1024"] = cpu_chain_baseline(out.get("chain1024"))

    print(json.dumps(out), flush=True)
    # the batch generator's worker pool is shut down by its with-block; make
    # sure no child process outlives the run
    import multiprocessing
    for ch in multiprocessing.active_children():
        ch.join(timeout=10)


GEMM_SOURCES = ("paper_2005_10680_amd/csrc/gemm.hip", "paper_2005_10680_amd/csrc/kernels.hpp",
                "paper_2005_10680_amd/csrc/common.hpp")


def gemm_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in GEMM_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def product_kernel_stats(precision, b, pairs, low, gemm_ms, launches):
    """The leaf-product kernel of one purification, from its stream-event
    times: the operands its kept pairs stream through the CUs (2 b^2 values
    per pair: 8 B each for an FP64 pair, 4 B for an FP32 one, 2 x 2 B for a
    split-BF16 one), and the fraction of the MFMA peaks its flops would need
    (FP64 pairs 2b^3 at 78.6 TFLOP/s; FP32 pairs 2b^3 at 157.3; split-BF16
    pairs 3 x 2b^3 at 2.5 PFLOP/s)."""
    s = gemm_ms / 1e3
    f64 = pairs - low
    low_bytes = {"fp64": 8, "fp32": 4, "bf16x3": 4}[precision]
    stream = (f64 * 8 + low * low_bytes) * 2.0 * b * b
    t_peak = f64 * 2.0 * b ** 3 / 78.6e12
    if precision == "fp32":
        t_peak += low * 2.0 * b ** 3 / 157.3e12
    elif precision == "bf16x3":
        t_peak += low * 3 * 2.0 * b ** 3 / 2.5e15
    kern = {"fp64": f"k_gemm_ring<{b},0>", "fp32": f"k_gemm_ring<{b},1>", "bf16x3": f"k_gemm_ring<{b},2>"}[precision]
    return {"kernel": kern, "ms_per_launch": round(gemm_ms / max(launches, 1), 4),
            "operand_stream_GB_per_s": round(stream / s / 1e9, 1),
            "operand_stream_frac_of_hbm_peak": round(stream / s / 8e12, 4),
            "mfma_frac_at_the_peaks": round(t_peak / s, 4)}


def measured_traffic(n, b, seed):
    """HBM bytes per launch of the leaf-product kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary of this workload, each counter scaled by
    what it reads for a plain 1 GiB device copy.  None when no summary exists
    or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_gemm_ring_f64_sys3d_n{n}_s{seed}_leaf{b}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", " ", "\t")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != gemm_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def adjoint_leg(dev, P, synth, torch):
    """Reverse mode of the purification of the 3D system n = 32768 (seed 5,
    leaf 64) for L = <D~, W>, W symmetric banded (bandwidth 64, N(0,1)
    entries, seed 55): forward with checkpoints every 8 iterates, then
    purify_sp2_adjoint (segments recomputed).  Without a dense spectrum at
    this size the per-step delta is a constant (1e-9).  Checked against
    central differences of L along a random symmetric direction H on F's
    pattern, with the perturbed runs' decisions compared to the base run's
    (equal decisions: the frozen map is the map that ran)."""
    n, b, seed, every, nmax = 32768, 64, 5, 8, 60
    taus = synth.tau_log(32)
    eps, dconst = 1e-6, 1e-9
    t0 = time.perf_counter()
    Fh = synth.sys3d(n, seed, b)
    Wh = synth.band_w(n, b, 64, 55)
    Uh = synth.symmetric_direction(n, b, Fh, 7)
    log(f"adjoint: inputs n={n} generated in {time.perf_counter() - t0:.1f} s")
    F = P.BlockSparse.from_host(Fh)
    W = P.BlockSparse.from_host(Wh)
    # relative direction H = F * U (U symmetric, entries in (-1, 1)): zeros
    # stay zero and tiny entries move by tiny amounts, so the run's
    # decisions can stay those of the base run
    H = (torch.from_numpy(np.ascontiguousarray(Uh.vals).reshape(-1)).to(dev) *
         torch.from_numpy(np.ascontiguousarray(Fh.vals).reshape(-1)).to(dev))
    nb = F.nb
    kw = dict(delta_const=dconst, n_max=nmax)

    def loss_and_dbar(D):
        cap = D.cap
        nsl = int(D.nslot.item())
        brow = D.brow.long()
        bcol = D.bcol.long()
        live = (torch.arange(cap, device=dev) < nsl) & (brow >= 0)
        key = torch.where(live, brow * nb + bcol, torch.zeros_like(brow))
        ws_ = torch.where(live, W.map.long()[key], torch.full_like(brow, -1))
        Dv = D.val.view(cap, b * b)
        dbar = torch.zeros_like(Dv)
        m = ws_ >= 0
        dbar[m] = W.val.view(-1, b * b)[ws_[m]]
        return float((Dv * dbar).sum().item()), dbar.view(-1)

    P.purify(F, n // 2, eps, taus, **kw)          # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = P.purify(F, n // 2, eps, taus, keep_tape=every, **kw)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    L0, dbar = loss_and_dbar(res.D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fbar = P.purify_adjoint(res, F, dbar)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    got = float((fbar * H).sum().item())
    base = [(l["branch"], l["idx"], l["npairs"], l["nslot_kept"], l["removed_units"]) for l in res.logs]
    steps = sum(1 for l in res.logs if l["branch"] >= 0)
    status = res.status
    pairs = sum(l["npairs"] for l in res.logs if l["branch"] >= 0)
    log(f"adjoint: {steps} steps, forward with checkpoints {t_fwd:.3f} s, adjoint {t_adj:.3f} s")
    del res, dbar
    torch.cuda.empty_cache()
    fd = {}
    for h in (1e-5, 1e-6):
        vals, ndiff, maxdp, nrec = [], 0, 0, []
        for sgn in (1.0, -1.0):
            Fp = P.with_values(F, F.val + sgn * h * H)
            rp = P.purify(Fp, n // 2, eps, taus, **kw)
            mine = [(l["branch"], l["idx"], l["npairs"], l["nslot_kept"], l["removed_units"]) for l in rp.logs]
            nrec.append(len(mine))
            for a, c in zip(base, mine):
                if a != c:
                    ndiff += 1
                    maxdp = max(maxdp, abs(a[2] - c[2]))
            vals.append(loss_and_dbar(rp.D)[0])
            del rp, Fp
        d = (vals[0] - vals[1]) / (2.0 * h)
        fd[str(h)] = {"fd": d, "rel_diff": abs(d - got) / max(abs(d), 1e-300),
                      "records_base_plus_minus": [len(base)] + nrec,
                      "steps_with_other_decisions": ndiff, "max_kept_pair_difference": maxdp}
        log(f"adjoint: h={h:g} central difference {d:.9e} vs <Fbar, H> {got:.9e}; records {len(base)} vs {nrec}, "
            f"{ndiff} common steps with other decisions (kept pairs differ by at most {maxdp})")
    return {"workload": f"sys3d_n{n}_s{seed}_leaf{b}_bandW64", "steps": steps, "status": int(status),
            "kept_pairs_forward": int(pairs),
            "checkpoint_every": every, "delta_const": dconst, "loss": L0,
            "forward_with_checkpoints_s": round(t_fwd, 4), "adjoint_s": round(t_adj, 4),
            "directional_derivative": got, "central_differences": fd}


def candidate_list_leg(run_once, torch, reps, b, synth):
    """The main workload with other candidate lists: N log-spaced thresholds
    from 1 down to 1e-16 (N = 16, 32, 64, 128), and 40 from 1e4 (a first
    candidate above every block-pair product), in FP64 and, for N = 32 and
    64, the split-BF16 tier; time to D~ (median of reps), kept pairs, the
    sweep's share.  The selection rule and the error guarantee are the same
    for every list; a denser list lets tau (and sigma) sit closer to the
    budget at a higher sweep cost."""
    lists = [(f"log{N}", synth.tau_log(N)) for N in (16, 32, 64, 128)]
    lists.append(("log40_from_1e4", np.logspace(4.0, -16.0, 40)))
    rows = []
    for name, taus_ in lists:
        for prec in ("fp64", "bf16x3"):
            if prec != "fp64" and name not in ("log32", "log64"):
                continue
            t, r = timed(lambda: run_once(prec, taus_=taus_), torch, reps)
            st = [lg for lg in r.logs if lg["branch"] >= 0]
            rows.append({"list": name, "N": int(len(taus_)), "precision": prec, "sp2_time_s": round(t, 4),
                         "iterations": len(st), "kept_pairs_per_run": int(sum(lg["npairs"] for lg in st)),
                         "low_tier_pairs_per_run": int(sum(lg["npairs_low"] for lg in st)),
                         "sweep_ms_per_run": round(sum(lg["ms_sweep"] for lg in st), 3)})
            log(f"candidates {name} ({prec}): {t:.3f} s, {rows[-1]['kept_pairs_per_run']} kept pairs, "
                f"sweep {rows[-1]['sweep_ms_per_run']:.1f} ms")
            del r
    return rows


def variants_leg(run_once, torch, reps, b, eps, verify_err):
    """The purification of the main workload with each of the paper's
    variants: Algorithm 5 (hybrid: SpAMM with delta_i/2, truncation with
    delta_i/2), Algorithm 4 (SpAMM with delta_i, no truncation) and
    Algorithm 1 (exact product, truncation with delta_i).  Per variant: time
    to D~ (median of reps host-loop runs), iterations, per-iteration mean of
    the threshold sweep (T_CSE), the product (T_SpAMM, or T_mul for
    Algorithm 1: kept-pair list and leaf products) and the truncation
    (T_trunc), the mean and largest block counts of X^_i and X~_i, and
    ||D - D~||_F against eps."""
    rows = {}
    for v in ("hybrid", "spamm", "truncmul"):
        run_once(variant=v)
        t, r = timed(lambda: run_once(variant=v), torch, reps)
        st = [lg for lg in r.logs if lg["branch"] >= 0]
        it = max(len(st), 1)
        pairs = sum(lg["npairs"] for lg in st)
        rows[v] = {"algorithm": {"hybrid": 5, "spamm": 4, "truncmul": 1}[v], "sp2_time_s": round(t, 4),
                   "iterations": len(st), "kept_pairs_per_run": int(pairs),
                   "kept_TFLOP_per_s": round(pairs * 2.0 * b ** 3 / t / 1e12, 3),
                   "ms_per_iteration": {
                       "cse": round(sum(lg["ms_sweep"] for lg in st) / it, 4),
                       "product": round(sum(lg["ms_pairs"] + lg["ms_gemm"] + lg["ms_norms"] for lg in st) / it, 4),
                       "trunc": round(sum(lg["ms_trunc"] for lg in st) / it, 4),
                       "total": round(sum(lg["ms_total"] for lg in st) / it, 4)},
                   "blocks_Xhat_mean_max": [round(float(np.mean([lg["nslot_hat"] for lg in st])), 1),
                                            int(max(lg["nslot_hat"] for lg in st))],
                   "blocks_Xtilde_mean_max": [round(float(np.mean([lg["nslot_kept"] for lg in st])), 1),
                                              int(max(lg["nslot_kept"] for lg in st))],
                   "status": int(r.status), "eps": eps, "verify_fro_err": verify_err(r)}
        log(f"variant {v}: {t:.3f} s, {len(st)} iterations, {pairs} kept pairs, "
            f"err {rows[v]['verify_fro_err']}")
        del r
        torch.cuda.empty_cache()
    return rows


def fro_diff(A, B, torch):
    """||A - B||_F of two device block-sparse matrices of the same shape and
    leaf size (block-wise over the union of their patterns)."""
    b, nb = A.b, A.nb
    bb = b * b

    def live(M):
        ns = min(int(M.nslot.item()), M.cap)
        br, bc = M.brow[:ns].long(), M.bcol[:ns].long()
        ok = br >= 0
        return torch.nonzero(ok).flatten(), (br * nb + bc)[ok]

    sa, ka = live(A)
    sb, kb = live(B)
    va = A.val.view(-1, bb)
    vb = B.val.view(-1, bb)
    tot = 0.0
    chunk = 1 << 14
    for q in range(0, sa.shape[0], chunk):
        s_a, k_a = sa[q:q + chunk], ka[q:q + chunk]
        m_b = B.map[k_a].long()
        other = torch.where((m_b >= 0)[:, None], vb[m_b.clamp(min=0)], torch.zeros((), dtype=va.dtype, device=va.device))
        tot += float(((va[s_a] - other) ** 2).sum().item())
    for q in range(0, sb.shape[0], chunk):
        s_b, k_b = sb[q:q + chunk], kb[q:q + chunk]
        only = A.map[k_b].long() < 0
        if bool(only.any()):
            tot += float((vb[s_b[only]] ** 2).sum().item())
    return math.sqrt(tot)


def norms_rate(M, b, reps=10):
    """HBM rate of the stand-alone norms kernel over the live blocks of M
    (stream events around reps calls on the library's stream)."""
    import torch
    import paper_2005_10680_amd as P
    P.build_norms(M)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.build_norms(M)
    e1.record()
    torch.cuda.synchronize()
    r = hbm_rate(live_blocks(M) * 8.0 * b * b, e0.elapsed_time(e1) / reps)
    r["blocks"] = live_blocks(M)
    return r


def hbm_rate(nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bytes_per_run": nbytes, "ms_per_run": round(ms, 3), "achieved_GB_per_s": round(gbs, 1),
            "peak_GB_per_s": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4)}


def live_blocks(M):
    ns = min(int(M.nslot.item()), M.cap)
    return int((M.brow[:ns] >= 0).sum().item())


def timed(fn, torch, reps):
    """(median seconds, last result) of fn() with device syncs around each call."""
    ts, r = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), r


def protocol_leg(P, torch, D, taus, deltas=(1e-6, 1e-8, 1e-10), reps=3):
    """The paper's multiplication experiment on a converged density matrix:
    C~ = SpAMM(D~, D~) with tau from the sweep for each error budget delta,
    against the exact product (tau = 0) followed by truncation at delta.
    Times are whole library calls (sweep / multiply / truncate), median of
    reps; reports whether the measured error ||C~ - D~^2||_F sits below the
    bound and below delta."""
    b = D.b
    P.build_norms(D)
    nb = D.nb
    Cx = P.BlockSparse(D.n, b, nb * nb, D.device)
    t_mul, r = timed(lambda: P.multiply(D, D, 0.0, symmetric=True, b_transposed=True, out=Cx), torch, reps)
    all_pairs = int(r[1][0].item())
    nnz_exact = live_blocks(Cx)
    Ca = P.BlockSparse(D.n, b, nb * nb, D.device)
    Ct = P.BlockSparse(D.n, b, nb * nb, D.device)
    rows = []
    for delta in deltas:
        t_cse, (bound, idx, tau) = timed(lambda: P.sweep_tau(D, D, taus, delta, b_transposed=True), torch, reps)
        m = int(idx.item())
        tau_v = float(tau.item())
        bnd = float(bound[m].item()) if m < len(taus) else 0.0
        flat = P.sweep_tau(D, D, taus, delta, b_transposed=True, bound="flat")
        t_sp, r = timed(lambda: P.multiply(D, D, tau_v, symmetric=True, b_transposed=True, out=Ca), torch, reps)
        kept = int(r[1][0].item())
        err = fro_diff(Ca, Cx, torch)

        # time only the truncation call, on a fresh copy of the exact product each time
        tt = []
        for _ in range(reps):
            ns = int(Cx.nslot.item())
            for a in ("nslot", "brow", "bcol", "map"):
                getattr(Ct, a).copy_(getattr(Cx, a))
            Ct.val[: ns * b * b].copy_(Cx.val[: ns * b * b])
            P.build_norms(Ct)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.truncate(Ct, delta, sync=True)
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t0)
        t_tr = float(np.median(tt))
        err_tr = fro_diff(Ct, Cx, torch)
        rows.append({"delta": delta, "tau": tau_v, "bound": bnd, "err_measured": err,
                     "tau_flat": float(flat[2].item()), "kept_pairs": kept, "all_pairs": all_pairs,
                     "nnz_spamm": live_blocks(Ca), "nnz_trunc": live_blocks(Ct), "nnz_exact": nnz_exact,
                     "ms_cse": round(1e3 * t_cse, 3), "ms_spamm": round(1e3 * t_sp, 3),
                     "ms_mul": round(1e3 * t_mul, 3), "ms_trunc": round(1e3 * t_tr, 3),
                     "err_trunc": err_tr,
                     "spamm_kept_TFLOP_per_s": round(kept * 2.0 * b ** 3 / t_sp / 1e12, 3)})
        log(f"protocol delta={delta:.0e}: tau={tau_v:.3e} kept {kept}/{all_pairs} err {err:.3e} <= bound "
            f"{bnd:.3e}; cse {1e3 * t_cse:.2f} ms, spamm {1e3 * t_sp:.2f} ms, mul {1e3 * t_mul:.2f} ms, "
            f"trunc {1e3 * t_tr:.2f} ms")
        rows[-1]["err_below_bound"] = bool(err <= bnd or err < 1e-300)
        rows[-1]["err_below_delta"] = bool(err < delta)
        # the hybrid step (Algorithm 5): SpAMM with delta/2, then truncation with delta/2
        t_cse_h, (_, idx_h, tau_h) = timed(lambda: P.sweep_tau(D, D, taus, delta / 2, b_transposed=True), torch,
                                           reps)
        tau_hv = float(tau_h.item())
        t_sp_h, r = timed(lambda: P.multiply(D, D, tau_hv, symmetric=True, b_transposed=True, out=Ca), torch, reps)
        kept_h = int(r[1][0].item())
        nnz_hat = live_blocks(Ca)
        tt = []
        for _ in range(reps):
            ns = int(Ca.nslot.item())
            for a in ("nslot", "brow", "bcol", "map"):
                getattr(Ct, a).copy_(getattr(Ca, a))
            Ct.val[: ns * b * b].copy_(Ca.val[: ns * b * b])
            P.build_norms(Ct)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.truncate(Ct, delta / 2, sync=True)
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t0)
        err_h = fro_diff(Ct, Cx, torch)
        rows[-1]["hybrid"] = {"tau": tau_hv, "kept_pairs": kept_h, "nnz_hat": nnz_hat, "nnz_tilde": live_blocks(Ct),
                              "ms_cse": round(1e3 * t_cse_h, 3), "ms_spamm": round(1e3 * t_sp_h, 3),
                              "ms_trunc": round(1e3 * float(np.median(tt)), 3), "err_measured": err_h,
                              "err_below_delta": bool(err_h < delta)}
        log(f"protocol delta={delta:.0e} hybrid: tau={tau_hv:.3e} kept {kept_h}, blocks {nnz_hat} -> "
            f"{live_blocks(Ct)}, err {err_h:.3e}")
    del Cx, Ca, Ct
    torch.cuda.empty_cache()
    return rows


def chain_leg(P, torch, synth, reps=20):
    """The small chain workload (n = 1024, leaf 32, the paper's 350
    candidates, seed 1): a few hundred kept pairs per step, so the host
    loop's per-step launches and read-backs dominate; timed with the host
    loop and with the graph-captured loop (poll every 8 steps), median of
    reps, with the spectrum's gap from the committed dense eigenvalues."""
    spec = load_spectrum("chain1d_n1024_s1_b32")
    Fh = synth.chain1d(1024, 1, 32)
    F = P.BlockSparse.from_host(Fh)
    taus = torch.as_tensor(synth.tau_paper(), dtype=torch.float64, device=F.device)  # resident, like F
    kw = dict(homo=spec["homo"], lumo=spec["lumo"])
    host = lambda: P.purify(F, 512, 1e-6, taus, **kw)
    graph = lambda: P.purify(F, 512, 1e-6, taus, graph_steps=8, **kw)
    host()
    graph()
    th, rh = timed(host, torch, reps)
    tg, rg = timed(graph, torch, reps)
    st = [lg for lg in rh.logs if lg["branch"] >= 0]
    same = [lg["npairs"] for lg in rg.logs] == [lg["npairs"] for lg in rh.logs]
    log(f"chain n=1024: host loop {1e3 * th:.2f} ms, graph loop {1e3 * tg:.2f} ms, {len(st)} iterations")
    return {"workload": "sp2_hybrid_chain1d_n1024_leaf32_tau350_eps1e-6", "iterations": len(st),
            "kept_pairs_per_run": int(sum(lg["npairs"] for lg in st)),
            "host_loop_ms": round(1e3 * th, 3), "graph_loop_ms": round(1e3 * tg, 3),
            "graph_speedup": round(th / tg, 3), "same_decisions": bool(same)}


def big_leg(P, torch, synth, reps=1):
    """The 65536 workload (3D system, seed 3, leaf 64): time to D~ in FP64
    and with the FP32 and split-BF16 leaf-product tiers (Algorithm 3's
    bound), and in FP64 and split BF16 selecting with B_flat, each D~ compared
    with a reference run of the FP64 path at a 100 times smaller per-step
    delta (no dense eigensolver at this size; the per-step delta is a
    constant, 1e-9)."""
    n, b, seed = 65536, 64, 3
    t0 = time.perf_counter()
    Fh = synth.sys3d(n, seed, b)
    log(f"big: input n={n} generated in {time.perf_counter() - t0:.1f} s ({Fh.nblk} blocks)")
    F = P.BlockSparse.from_host(Fh)
    del Fh
    taus = synth.tau_log(32)
    nb = F.nb
    n_occ = n // 2

    def run(precision, dconst, bound="tree"):
        return P.purify(F, n_occ, 1e-6, taus, delta_const=dconst, cap=nb * nb, precision=precision, bound=bound)

    def keep_d(res):
        """A compact device copy of the result (only its live slots)."""
        D = res.D
        ns = int(D.nslot.item())
        K = P.BlockSparse(n, b, max(ns, 1), D.device)
        K.nslot.copy_(D.nslot)
        K.brow.copy_(D.brow[:K.cap])
        K.bcol.copy_(D.bcol[:K.cap])
        K.map.copy_(D.map)
        K.val.copy_(D.val[: K.cap * b * b])
        return K

    ref = run("fp64", 1e-11)
    rsteps = [lg for lg in ref.logs if lg["branch"] >= 0]
    Dref = keep_d(ref)
    del ref
    torch.cuda.empty_cache()
    log(f"big: reference run done, {len(rsteps)} iterations")
    out = {"workload": f"sp2_hybrid_sys3d_n{n}_leaf{b}_tau32_eps1e-6_seed{seed}", "delta_const": 1e-9,
           "reference": {"delta_const": 1e-11, "iterations": len(rsteps),
                         "kept_pairs": int(sum(lg["npairs"] for lg in rsteps))}}
    base_t = None
    for prec, bound in (("fp64", "tree"), ("fp32", "tree"), ("bf16x3", "tree"), ("fp64", "flat"),
                        ("bf16x3", "flat")):
        key = prec if bound == "tree" else f"{prec}_flat"
        run(prec, 1e-9, bound)                  # warm-up
        t, r = timed(lambda: run(prec, 1e-9, bound), torch, reps)
        st = [lg for lg in r.logs if lg["branch"] >= 0]
        pairs = sum(lg["npairs"] for lg in st)
        low = sum(lg["npairs_low"] for lg in st)
        err = fro_diff(r.D, Dref, torch)
        base_t = t if key == "fp64" else base_t
        out[key] = {"bound": bound, "sp2_time_s": round(t, 4), "iterations": len(st), "kept_pairs": int(pairs),
                     "low_tier_pairs": int(low), "kept_TFLOP_per_s": round(pairs * 2.0 * b ** 3 / t / 1e12, 3),
                     "fro_err_vs_reference": err, "peak_blocks": int(max(lg["nslot_hat"] for lg in st)),
                     "speedup_vs_fp64": round(base_t / t, 4),
                     "phase_ms": {k: round(sum(lg[k] for lg in st), 2)
                                  for k in ("ms_sweep", "ms_pairs", "ms_gemm", "ms_norms", "ms_trunc")}}
        log(f"big {key}: {t:.3f} s, {len(st)} iterations, low-tier {low}/{pairs}, err vs reference {err:.3e}")
        del r
        torch.cuda.empty_cache()
    del Dref, F
    torch.cuda.empty_cache()
    return out


def _gen_leaf32(arg):
    n, seed = arg
    import synth
    return synth.sys3d(n, seed, 32)


def generate_batch(count, synth):
    """The first `count` systems of the batched workload at leaf 32 (process
    pool; called before any GPU use)."""
    from concurrent.futures import ProcessPoolExecutor
    sizes = synth.batch_sizes(4, 64)[:count]
    t0 = time.perf_counter()
    workers = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        mats = list(ex.map(_gen_leaf32, sizes))
    log(f"batch: generated {len(mats)} systems (sum n = {sum(n for n, _ in sizes)}) in {time.perf_counter() - t0:.1f} s")
    return mats


def batch_bytes(P, F, cap, max_pairs, taus, prec):
    """Device bytes one system adds to a batched call: its share of the
    workspace and its output matrix."""
    import ctypes
    p = P.sp2_params(F.n // 2, 1e-6, 60, 0, 0, len(taus), float("nan"), float("nan"), 1e-9, 0.0, 0,
                     P.PRECISIONS[prec], 0.5, 8, 0)
    ws = P.lib().purify_sp2_batched_workspace_bytes(1, ctypes.byref(F.struct()), ctypes.byref(p),
                                                    (ctypes.c_int64 * 1)(int(cap)),
                                                    (ctypes.c_int64 * 1)(int(max_pairs)))
    out = cap * (F.b * F.b * 8 + 4 * 8) + F.nb * F.nb * 4
    return float(ws + out)


def batch_leg(args, dev, P, synth, mats):
    """The batched workload: independent 3D systems (sizes log-uniform in
    [2048, 32768], generator seed 4, system seeds 4000 + s), generated at
    leaf 32, each re-blocked to the leaf size the autotuner picks for it,
    then purified together (one product launch per leaf size and tier per
    step, graph-captured loop) and, for comparison, one after another.
    Without dense spectra at these sizes the per-step delta is a constant
    (1e-9, the range the gap-based schedule gives for the n = 16384 system)."""
    import torch
    taus = synth.tau_log(32)
    eps, dconst = 1e-6, 1e-9
    saved = {b: P.get_gemm_schedule(b) for b in (32, 64, 128)}
    Fs, leaves = [], []
    t0 = time.perf_counter()
    for m in mats:
        F32 = P.BlockSparse.from_host(m)
        b, _, _ = P.autotune(F32, m.n // 2, eps, taus, delta_const=dconst, trial_steps=6)
        for bb, v in saved.items():
            P.set_gemm_schedule(bb, v)
        Fs.append(F32 if b == 32 else P.reblock(F32, b))
        leaves.append(b)
        del F32
        torch.cuda.empty_cache()
        if len(leaves) % 8 == 0:
            log(f"batch: autotuned {len(leaves)}/{len(mats)} systems")
    log(f"batch: autotuned leaf sizes {dict((b, leaves.count(b)) for b in sorted(set(leaves)))} "
        f"in {time.perf_counter() - t0:.1f} s")
    del mats
    res_all = {}
    caps_used = None
    for prec in ("fp64", "fp32"):
        if prec == "fp32" and any(b > 64 for b in leaves):
            continue
        # one after another (graph loop each, capacity nb^2): the comparison,
        # and the peak block count of every system (runs are deterministic,
        # so the batched run needs exactly these capacities)
        peaks, pair_peaks, ts = [], [], 0.0
        seq_logs = []
        for F in Fs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r1 = P.purify(F, F.n // 2, eps, taus, delta_const=dconst, precision=prec, graph_steps=8)
            torch.cuda.synchronize()
            ts += time.perf_counter() - t0
            nf = int(F.live()[0].shape[0])
            peaks.append(max([nf + F.nb] + [int(l["nslot_hat"]) for l in r1.logs]))
            pair_peaks.append(max([1] + [int(l["npairs"]) for l in r1.logs]))
            seq_logs.append([(l["branch"], l["idx"], l["npairs"]) for l in r1.logs])
            del r1
        torch.cuda.empty_cache()
        log(f"batch {prec}: one after another {ts:.3f} s (peak capacities measured)")
        caps = [min(F.nb * F.nb, pk) for F, pk in zip(Fs, peaks)]
        caps_used = caps
        # the systems go into as few batched calls as fit in free device memory
        # (workspace plus output, which doubles as the second iterate buffer)
        free, _ = torch.cuda.mem_get_info()
        budget = 0.8 * free
        chunks, cur, used = [], [], 0.0
        for q, (F, cp, mp) in enumerate(zip(Fs, caps, pair_peaks)):
            need = batch_bytes(P, F, cp, mp, taus, prec)
            if cur and used + need > budget:
                chunks.append(cur)
                cur, used = [], 0.0
            cur.append(q)
            used += need
        chunks.append(cur)

        def run_chunks():
            out_logs, out_status = [None] * len(Fs), [None] * len(Fs)
            for ch in chunks:
                kw = dict(delta_const=dconst, precision=prec, caps=[caps[q] for q in ch],
                          max_pairs=[pair_peaks[q] for q in ch], graph_steps=8, raise_on_error=False)
                r = P.purify_batched([Fs[q] for q in ch], [Fs[q].n // 2 for q in ch], eps, taus, float("nan"),
                                     float("nan"), **kw)
                for t, q in enumerate(ch):
                    out_logs[q], out_status[q] = r.logs[t], r.status[t]
                del r
            return out_logs, out_status
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        logs_b, status_b = run_chunks()
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        ok = sum(1 for st in status_b if st >= 0)
        same = all([(l["branch"], l["idx"], l["npairs"]) for l in lg] == sl for lg, sl in zip(logs_b, seq_logs))
        flops = sum(sum(l["npairs"] for l in lg if l["branch"] >= 0) * 2.0 * F.b ** 3 for lg, F in zip(logs_b, Fs))
        iters = [sum(1 for l in lg if l["branch"] >= 0) for lg in logs_b]
        torch.cuda.empty_cache()
        log(f"batch {prec}: {tb:.3f} s together ({len(chunks)} batched calls), {ts:.3f} s one by one, "
            f"{ok}/{len(Fs)} systems ok")
        res_all[prec] = {"time_s": round(tb, 4), "kept_TFLOP_per_s": round(flops / tb / 1e12, 4),
                         "batched_calls": len(chunks), "systems_per_call": [len(c) for c in chunks],
                         "sequential_time_s": round(ts, 4), "speedup_vs_sequential": round(ts / tb, 4),
                         "systems_ok": ok, "iterations_min_max": [min(iters), max(iters)],
                         "same_decisions_as_single_runs": bool(same)}
    dense = sum(F.nb * F.nb for F in Fs)
    gib = sum(cp * F.b * F.b * 8 for cp, F in zip(caps_used, Fs)) / 2 ** 30 if caps_used else None
    return {"systems": len(Fs), "iterate_capacity_GiB": round(gib, 2) if gib else None, "sum_n": int(sum(F.n for F in Fs)),
            "leaf_counts": {str(b): leaves.count(b) for b in sorted(set(leaves))},
            "capacity_fraction_of_dense": round(sum(caps_used) / dense, 4) if caps_used else None,
            "delta_const": dconst, **res_all}


def cpu_baseline(res, Fh, taus, b, seconds):
    """The oracle timed on the host cores on a bounded sample of the same
    workload: the last purification step's SpAMM (the sweep over the whole
    matrix, then the leaf products of a sample of output blocks)."""
    import oracle
    tape_X = res.D.to_host()
    X = oracle.BSM(tape_X.n, b, tape_X.brow, tape_X.bcol, tape_X.vals)
    t0 = time.perf_counter()
    _, nu = oracle.norms(X)
    bound = oracle.cse_tree(X, X, taus, nu, nu)
    steps = [l for l in res.logs if l["branch"] >= 0]
    budget = steps[-1]["delta"] / 2.0
    idx, tau = oracle.select(bound, taus, budget)
    K = oracle.kept(X, X, tau, True, nu, nu)
    t_sweep = time.perf_counter() - t0
    # sample outputs until about `seconds` of product work
    rng = np.random.default_rng(0)
    order = rng.permutation(K.oi.shape[0])
    pairs_per = (K.kptr[1:] - K.kptr[:-1])[order]
    done_pairs, done_s, pos = 0, 0.0, 0
    chunk = 64
    while done_s < seconds and pos < order.shape[0]:
        sel = order[pos:pos + chunk]
        t = time.perf_counter()
        oracle.block_products(X, X, K, sel)
        done_s += time.perf_counter() - t
        done_pairs += int(pairs_per[pos:pos + chunk].sum())
        pos = min(pos + chunk, order.shape[0])
        chunk = min(chunk * 2, 4096)
    tflops = done_pairs * 2.0 * b ** 3 / done_s / 1e12
    return {"value": tflops, "unit": "TFLOP/s", "cores": oracle_threads(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"last purification step of the same workload: exact-norm sweep over all "
                      f"{K.npairs} kept pairs ({t_sweep:.1f} s) and the leaf products of {pos} of "
                      f"{K.oi.shape[0]} output blocks ({done_pairs} pairs, {done_s:.1f} s)"}


def oracle_threads():
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:
        threads = min(threads, len(os.sched_getaffinity(0)))
    except AttributeError:
        pass
    return threads


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_chain_baseline(gpu_chain):
    """The oracle's whole purification of the small chain (n = 1024, leaf 32,
    the paper's 350 candidates, eps = 1e-6): every phase of every step on
    the host cores, against the GPU's time for the same run."""
    import oracle
    import synth
    spec = load_spectrum("chain1d_n1024_s1_b32")
    F = oracle.BSM.of(synth.chain1d(1024, 1, 32))
    p = oracle.SP2Params(n_occ=512, eps=1e-6, taus=synth.tau_paper(), homo=spec["homo"], lumo=spec["lumo"])
    t0 = time.perf_counter()
    _, logs, _ = oracle.sp2(F, p)
    t = time.perf_counter() - t0
    st = [lg for lg in logs if lg.branch >= 0]
    pairs = sum(lg.npairs for lg in st)
    out = {"value": round(t, 4), "unit": "s to D~ (whole purification)", "cores": oracle_threads(),
           "cpu_model": cpu_model(), "kind": "oracle", "iterations": len(st), "kept_pairs": int(pairs),
           "sample": "the whole chain purification (n = 1024, leaf 32, 350 candidates), every phase"}
    if gpu_chain:
        out["gpu_host_loop_s"] = gpu_chain["host_loop_ms"] * 1e-3
        out["gpu_graph_loop_s"] = gpu_chain["graph_loop_ms"] * 1e-3
        out["same_iterations_as_gpu"] = bool(len(st) == gpu_chain["iterations"])
        out["same_kept_pairs_as_gpu"] = bool(int(pairs) == gpu_chain["kept_pairs_per_run"])
    log(f"oracle chain purification: {t:.2f} s, {len(st)} iterations")
    return out


if __name__ == "__main__":
    main()
