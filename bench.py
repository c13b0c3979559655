#!/usr/bin/env python3
"""Throughput of the multi-determinant table method on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp64,mixed]
                    [--rows cfg3_fp64,...]

Headline workload: the water-like batched system -- 5 up + 5 down
electrons, 5 occupied + 20 virtual orbitals per spin from 40 s-Gaussians on
the three water nuclei, 10 000 determinants of orders 1-4, 4096 walkers, all
inputs seeded and synthetic.  One step is one sweep: every electron proposes
one move (ratio, gradient and laplacian of every determinant for every
walker) and the seeded 50 % acceptance mask commits it; the state is
recomputed from scratch once per sweep.  The K timed sweeps run as one HIP
graph with all inputs resident in device memory.

Metric: walker.det/s = walkers x determinants x moves / time.  The JSON line
also carries the roofline of the determinant kernel (bound by HBM: it streams
every walker's CI weights once per move; its FP64 vector-ALU figure beside),
the CPU oracle timed on a bounded sample of the same workload, and the other
precision forms.  Under "rows" (default: all of them) the other workloads of
the path, each with its own roofline block and oracle baseline:

* cfg3_*: molecular-shaped, n = 32 per spin, m = 224, 100 000 determinants,
  2048 walkers, in the FP64 form and the FP32-table forms, with the error of
  every output against stored oracle values (32 walkers x 10 moves);
* cfg4_adjoint: forward from the tables + backward, 1024 walkers, FP64;
* cfg5_uneven_*: 64 instances of uneven size (n = 5..64 per spin, m = 4n,
  10^2..2x10^5 determinants, 256 walkers each) moved together, FP64 and the
  rank-one FP32-table form.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6   # MI355X, 256 CUs x 2.4 GHz x 128 FP64 flop/clk/CU
PEAK_HBM_GBS = 8000.0

# FP64 flops of one excitation of order k in the determinant kernel
# (determinant, y = adj(S) c', four bordered derivative terms, five CI
# accumulations), counted from the kernel's closed-form small determinants
# of orders 1-4; FMA counts 2.
DET_FLOPS = {1: 26, 2: 43, 3: 80, 4: 165}


def det_flops(k: int) -> int:
    if k in DET_FLOPS:
        return DET_FLOPS[k]
    # generic path: k+1 eliminations of k x k (2k^3/3 each) + 4(2k+2) + 10
    return int((k + 1) * 2 * k ** 3 / 3 + 4 * (2 * k + 2) + 10)


def flops_per_launch(exc, W: int) -> float:
    orders = exc.orders()
    return float(W) * sum(det_flops(int(k)) for k in orders if k > 0)


def bytes_per_launch(exc, W: int, n: int, m: int, precision: str, fused: bool = True) -> float:
    """Algorithmic HBM bytes of one determinant-kernel launch: each walker's CI
    weight C_u of every excitation of the moving spin (8 B, read once), the
    walker's inputs once and its output sums once.  FP64 form with the
    proposal formed in the kernel (n <= 8): T [n*m], the inverse [n*n], the
    new orbital values and their gradient and laplacian [5(n+m)], six sums
    out.  FP64 form with a separate proposal kernel: T [n*m], the e-terms
    [5m], c [n], six sums out.  FP32-table forms: T' [n*m], g^a [4m], c' [n]
    in FP32, five sums out."""
    U = int((exc.orders() > 0).sum())
    if precision == "fp64":
        if fused:
            return float(W) * (8 * U + 8 * (n * m + n * n + 5 * (n + m)) + 6 * 8)
        return float(W) * (8 * U + 8 * (n * m + 5 * m + n) + 6 * 8)
    return float(W) * (8 * U + 4 * (n * m + 4 * m + n) + 5 * 8)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_det_propose_water_batched_traffic.md")
KERNEL_SOURCES = ("paper_1106_2456_amd/csrc/k_dets.hip", "paper_1106_2456_amd/csrc/mde_internal.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(plan):
    """HBM bytes per launch of the determinant kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter
    on a copy of known size), or None when the kernel sources or the plan
    have changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if line.startswith("traffic_"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("traffic_source_hash") != kernel_source_hash():
        return None
    if kv.get("traffic_plan") != json.dumps(plan, sort_keys=True):
        return None
    return float(kv["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_context(wl, precision, stream, refresh_every):
    from paper_1106_2456_amd import Context
    s = wl.system
    W = wl.walkers.W
    ctx = Context(s.n_elec, s.n_orb, W, max_order=4, refresh_every=refresh_every,
                  precision=precision, stream=stream)
    ctx.set_expansion(s.exc[0], s.exc[1], s.coef, s.det_up, s.det_dn)
    for sp in (0, 1):
        ctx.set_basis(sp, s.centres, s.expo, s.mo_spin(sp))
    ctx.bind(W)
    return ctx


def run_form(wl, precision, steps, warmup, autotune=True, repeat=8, check=None):
    """Time `steps` sweeps (one graph) of one precision form; returns a dict.
    check(ctx) runs first on the bound context (e.g. a parity replay) and its
    result is returned under "check"."""
    import torch
    s = wl.system
    W = wl.walkers.W
    n_tot = s.n_elec[0] + s.n_elec[1]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = build_context(wl, precision, stream, refresh_every=n_tot)
        checked = check(ctx) if check is not None else None
        pos = torch.as_tensor(wl.walkers.pos, device="cuda")
        nu = s.n_elec[0]
        ou = ctx.sgauss_eval(0, pos[:, :nu].contiguous())
        od = ctx.sgauss_eval(1, pos[:, nu:].contiguous())
        ctx.init(ou, od)
        # inputs of one sweep, resident in device memory
        moves = []
        for k in range(n_tot):
            e = int(wl.moves.electron[k])
            new_r = torch.as_tensor(wl.walkers.pos[:, e] + wl.moves.disp[k], device="cuda")
            moves.append((e, ctx.sgauss_eval(ctx.spin_of(e), new_r.contiguous()),
                          torch.as_tensor(wl.moves.accept_half[k], dtype=torch.uint8, device="cuda")))
        outs = [(torch.empty(W, dtype=torch.float64, device="cuda"),
                 torch.empty((W, 3), dtype=torch.float64, device="cuda"),
                 torch.empty(W, dtype=torch.float64, device="cuda"),
                 torch.zeros(W, dtype=torch.int32, device="cuda")) for _ in range(n_tot)]
        if autotune:
            up = next(m[1] for m in moves if m[0] < nu)
            dn = next(m[1] for m in moves if m[0] >= nu)
            ctx.autotune(up, dn)
            ctx.init(ou, od)
        plan = [ctx.get_plan(0), ctx.get_plan(1)]

        def sweep():
            for (e, no, mask), out in zip(moves, outs):
                ctx.propose(e, no, out)
                ctx.accept(e, mask)

        # warmup graph and timed graph (K sweeps in one graph)
        stream.synchronize()
        with ctx.capture() as cw:
            for _ in range(max(warmup, 1)):
                sweep()
        with ctx.capture() as ct:
            for _ in range(steps):
                sweep()
        for _ in range(1 if warmup > 0 else 0):
            cw.graph.launch()
        stream.synchronize()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        ct.graph.launch()
        t1.record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        ms_total = t0.elapsed_time(t1)
        # the same K sweeps issued directly (no graph)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            sweep()
        e1.record(stream)
        stream.synchronize()
        ms_eager = e0.elapsed_time(e1)
        # K more sweeps with a HIP event pair on the context's stream around
        # every launch of the determinant kernel (events recorded inside a
        # graph carry no timestamps on this runtime): once with one launch
        # per pair, once with `repeat` back-to-back launches per pair, which
        # spreads the dispatch gap after the first event over the repeats
        det = {}
        for rep in (1, repeat):
            ctx.profile_enable(steps * n_tot, rep)
            for _ in range(steps):
                sweep()
            stream.synchronize()
            det[rep] = ctx.profile_read()
            ctx.profile_disable()
        det_ms, det_n = det[repeat]
        single_ms, single_n = det[1]
        st = torch.stack([o[3] for o in outs]).cpu().numpy()
    ms_step = ms_total / steps
    wdets = W * s.n_det * n_tot
    fl = np.mean([flops_per_launch(s.exc[ctx.spin_of(m[0])], W) for m in moves])
    fused = precision == "fp64" and plan[0]["walker_tile"] == 64 and max(s.n_elec) <= 8
    by = np.mean([bytes_per_launch(s.exc[sp], W, s.n_elec[sp], s.n_orb[sp] - s.n_elec[sp], precision,
                                   fused)
                  for sp in (ctx.spin_of(m[0]) for m in moves)])
    det_avg_s = det_ms / max(det_n, 1) / 1e3
    return dict(precision=precision, ms_per_step=ms_step, value=wdets / (ms_step / 1e3),
                ms_per_step_eager=ms_eager / steps,
                det_launches=det_n, det_avg_us=det_avg_s * 1e6, det_flops_per_launch=fl,
                det_single_us=single_ms / max(single_n, 1) * 1e3, det_repeat=repeat,
                det_bytes_per_launch=by,
                det_gbs=by / det_avg_s / 1e9 if det_n else None,
                det_tflops=fl / det_avg_s / 1e12 if det_n else None, plan=plan,
                status_bits=int(np.bitwise_or.reduce(st.ravel())) if st.size else 0,
                check=checked)


def cpu_baseline(wl, target_seconds=12.0, probe=64, max_moves=None):
    """The oracle on a bounded sample of the same workload (the first walkers,
    the first moves of the sweep), on the host cores; max_moves=1: the first
    move of the first `probe` walkers."""
    import oracle
    s = wl.system
    threads = oracle.num_threads()
    n_tot = sum(s.n_elec)
    # size the walker sample so that one sweep takes about target_seconds
    probe = min(wl.walkers.W, probe)
    t0 = time.perf_counter()
    e = int(wl.moves.electron[0])
    oracle.move(s, wl.walkers.pos[:probe].copy(), e, wl.walkers.pos[:probe, e] + wl.moves.disp[0, :probe])
    dt_probe = time.perf_counter() - t0
    per_walker_move = dt_probe / probe
    if dt_probe > 0.5 * target_seconds or max_moves == 1:
        # one move of the probe sample is already the bounded sample
        return dict(value=probe * s.n_det / dt_probe, unit="walker.det/s", cores=threads,
                    kind="oracle",
                    sample=f"{probe} walkers x 1 move of the same workload "
                           f"(full-LU oracle, {dt_probe:.1f} s)")
    sample_w = int(min(wl.walkers.W, max(probe, target_seconds / (n_tot * per_walker_move))))
    pos = wl.walkers.pos[:sample_w].copy()
    moves = 0
    t0 = time.perf_counter()
    for k in range(n_tot):
        e = int(wl.moves.electron[k])
        oracle.move(s, pos, e, pos[:, e] + wl.moves.disp[k, :sample_w])
        moves += 1
        if time.perf_counter() - t0 > 3 * target_seconds:
            break
    dt = time.perf_counter() - t0
    walkers_done = moves * sample_w
    return dict(value=walkers_done * s.n_det / dt, unit="walker.det/s", cores=threads,
                kind="oracle",
                sample=f"{sample_w} walkers x {moves} moves of the same workload "
                       f"(full-LU oracle, {dt:.1f} s)")


def roofline_block(kernel, achieved_bytes, seconds, flops=None, traffic=None, note=None):
    """HBM roofline of one kernel from its algorithmic bytes per launch and its
    measured average launch time (FP64 vector-ALU figure beside)."""
    gbs = achieved_bytes / seconds / 1e9
    out = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": gbs / PEAK_HBM_GBS, "traffic": traffic, "kernel": kernel,
           "launch_us": seconds * 1e6, "bytes_per_launch": achieved_bytes}
    if flops is not None:
        tf = flops / seconds / 1e12
        out["alu"] = {"achieved": tf, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                      "frac": tf / PEAK_FP64_VECTOR_TFLOPS, "flops_per_launch": flops}
    if note:
        out["note"] = note
    return out


# ---- molecular-shaped rows (n = 32, m = 224, 100 000 determinants) -------------

GOLDEN_SCRIPT = os.path.join(ROOT, "tests", "golden", "make_molecular_sample.py")
MIXED_KIND = {"mixed": "round", "mixed_gemm": "gemm", "mixed_gemm_ksum64": "gemm"}


def golden_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_molecular_sample", GOLDEN_SCRIPT)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def molecular_workload():
    """Sweep workload of the molecular-shaped system (64 moves, every electron
    once) with the inputs the stored oracle sample was computed from."""
    gm = golden_module()
    g_wl, g = gm.load()
    wl = synth_mod().molecular(3, W=2048, n_det=100000, n_moves=64)
    wl.system = g_wl.system
    return wl, g_wl, g


def molecular_check(g_wl, g, precision):
    """Replay of the stored sample's 10 moves on the bound context: the error
    of every output of 32 walkers against the oracle's values (scaled as in
    the parity tests, and plain relative)."""
    import torch

    def check(ctx):
        pos = g_wl.walkers.pos.copy()
        nu = g_wl.system.n_elec[0]
        p = torch.as_tensor(pos, device="cuda")
        ctx.init(ctx.sgauss_eval(0, p[:, :nu].contiguous()), ctx.sgauss_eval(1, p[:, nu:].contiguous()))
        samp = g["sample"]
        scaled, plain = [], []
        for k, e in enumerate(g["electrons"]):
            e = int(e)
            new_r = pos[:, e] + g_wl.moves.disp[k]
            blk = ctx.sgauss_eval(ctx.spin_of(e), torch.as_tensor(new_r, device="cuda"))
            ratio, grad, lap, st = ctx.propose(e, blk)
            mask = g_wl.moves.accept_half[k]
            ctx.accept(e, torch.as_tensor(mask, dtype=torch.uint8, device="cuda"))
            got = np.column_stack([ratio.cpu().numpy()[samp], grad.cpu().numpy()[samp],
                                   lap.cpu().numpy()[samp]])
            ref = np.column_stack([g["ratio"][k], g["grad"][k], g["lap"][k]])
            if precision == "fp64":
                sc = np.column_stack([g["sc_ratio"][k], g["sc_grad"][k], g["sc_lap"][k]])
            else:
                sc = g["x_" + MIXED_KIND[precision]][k]
            d = np.abs(got - ref)
            scaled.append(d / sc)
            plain.append(d / np.abs(ref))
            acc = mask.astype(bool)
            pos[acc, e] = new_r[acc]
        scaled = np.concatenate(scaled)
        plain = np.concatenate(plain)
        out = {"sample": "32 walkers x 10 moves (both spins) against stored oracle values",
               "scale": "condition-aware" if precision == "fp64"
               else "first-order FP32-table-entry scale (" + MIXED_KIND[precision] + ")",
               "gate": 1e-10 if precision == "fp64" else 1e-5}
        for nm, c in (("ratio", slice(0, 1)), ("grad", slice(1, 4)), ("lap", slice(4, 5))):
            out[nm] = {"scaled_max": float(scaled[:, c].max()),
                       "plain_rel_max": float(plain[:, c].max()),
                       "plain_rel_median": float(np.median(plain[:, c])),
                       "plain_rel_above_1e-5": f"{int((plain[:, c] > 1e-5).sum())}/{plain[:, c].size}"}
        return out
    return check


def run_molecular(wl, g_wl, g, precision, steps, warmup, repeat=4):
    r = run_form(wl, precision, steps, warmup, autotune=True, repeat=repeat,
                 check=molecular_check(g_wl, g, precision))
    s = wl.system
    row = dict(value=r["value"], unit="walker.det/s", ms_per_step=r["ms_per_step"],
               ms_per_move=r["ms_per_step"] / sum(s.n_elec),
               workload=f"molecular-shaped: 32+32 electrons, 32+224 orbitals/spin, "
                        f"{s.n_det} determinants (orders 1-4), {wl.walkers.W} walkers, {precision}; "
                        "step = one sweep of 64 single-electron moves, 50% accepted",
               precision=precision, plan=r["plan"], status_bits=r["status_bits"],
               error=r["check"],
               roofline=roofline_block(f"k_det<{'double' if precision == 'fp64' else 'float'}, propose, "
                                       f"WT={r['plan'][0]['walker_tile']}>",
                                       r["det_bytes_per_launch"], r["det_avg_us"] * 1e-6,
                                       r["det_flops_per_launch"]))
    return row


def run_adjoint(steps, warmup, cpu=True):
    """Forward ln|sum_I c_I det S_up det S_dn| from the walkers' own tables and
    its adjoint (grad_c summed over walkers, grad_T per walker), FP64, on the
    water-like system with 1024 walkers; one step = eval_tables + backward."""
    import torch
    wl = synth_mod().water_like(4)
    s = wl.system
    W = wl.walkers.W
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = build_context(wl, "fp64", stream, refresh_every=None)
        pos = torch.as_tensor(wl.walkers.pos, device="cuda")
        nu = s.n_elec[0]
        ctx.init(ctx.sgauss_eval(0, pos[:, :nu].contiguous()), ctx.sgauss_eval(1, pos[:, nu:].contiguous()))
        Tu = ctx.export("table", 0).clone()
        Td = ctx.export("table", 1).clone()
        coef = torch.as_tensor(s.coef, device="cuda")
        go = torch.as_tensor(np.random.default_rng(44).normal(0, 1, W), device="cuda")

        def step():
            ctx.eval_tables(Tu, Td, coef)
            ctx.backward(go)

        for _ in range(max(warmup, 1)):
            step()
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / steps
        # the backward alone (its kernels run on the context's stream)
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        ctx.eval_tables(Tu, Td, coef)
        b0.record(stream)
        for _ in range(steps):
            ctx.backward(go)
        b1.record(stream)
        stream.synchronize()
        ms_bwd = b0.elapsed_time(b1) / steps
    # algorithmic HBM bytes of a step under this decomposition, per spin: the
    # table read and grad_T written (8 nm each), the ratios R written once
    # and read twice (CI precontraction gathers, coefficient gradient), the
    # CI weights C written once and read twice (N sum, table gradient)
    nm = [s.n_elec[sp] * (s.n_orb[sp] - s.n_elec[sp]) for sp in (0, 1)]
    U = [int((s.exc[sp].orders() > 0).sum()) + 1 for sp in (0, 1)]
    step_bytes = float(W) * sum(16 * nm[sp] + 48 * U[sp] for sp in (0, 1)) + 16.0 * s.n_det
    out = dict(value=W * s.n_det / (ms * 1e-3), unit="walker.det/s", ms_per_step=ms,
               ms_backward=ms_bwd,
               workload=f"water-like, {W} walkers, {s.n_det} determinants, FP64; "
                        "step = forward from the tables + backward (grad_c, grad_T)",
               roofline=roofline_block("adjoint step (eval_tables + backward, all kernels)",
                                       step_bytes, ms * 1e-3,
                                       note="bytes: T read and grad_T written, R written once "
                                            "and read twice, C written once and read twice, "
                                            "per spin; coef and grad_c"))
    if cpu:
        import oracle
        k = min(W, 256)
        tu, td = Tu[:k].cpu().numpy(), Td[:k].cpu().numpy()
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 8.0:
            oracle.tables(s, tu, td)
            reps += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=reps * k * s.n_det / dt, unit="walker.det/s",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"{k} walkers x {reps}, forward + adjoint by full LU "
                                          f"({dt:.1f} s)")
    return out


def run_local(wl, steps, cpu=True, tag="water-like"):
    """All-electron gradients and laplacians at fixed positions (one call of
    mde_local_derivs: every electron of every walker), FP64."""
    import torch
    s = wl.system
    W = wl.walkers.W
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = build_context(wl, "fp64", stream, refresh_every=None)
        pos = torch.as_tensor(wl.walkers.pos, device="cuda")
        nu = s.n_elec[0]
        ou = ctx.sgauss_eval(0, pos[:, :nu].contiguous())
        od = ctx.sgauss_eval(1, pos[:, nu:].contiguous())
        ctx.init(ou, od)
        out = ctx.local_derivs(ou, od)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            ctx.local_derivs(ou, od, out=out)
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1) / steps
    n_tot = sum(s.n_elec)
    # algorithmic bytes per call and spin: the CI weights (8 U), the table read
    # twice (8 nm each), dN/dT written and read (16 nm), the inverse (8 n^2),
    # every electron's four derivative rows (32 n (n + m)), outputs (32 n)
    byts = 0.0
    for sp in (0, 1):
        n, m = s.n_elec[sp], s.n_orb[sp] - s.n_elec[sp]
        U = int((s.exc[sp].orders() > 0).sum()) + 1
        byts += W * (8 * U + 32 * n * m + 8 * n * n + 32 * n * (n + m) + 32 * n)
    row = dict(value=W * s.n_det * n_tot / (ms * 1e-3), unit="walker.det.electron/s",
               ms_per_step=ms,
               workload=f"{tag}: all-electron grad ln Psi and lap Psi/Psi at fixed positions, "
                        f"{W} walkers, {s.n_det} determinants, {n_tot} electrons, FP64; "
                        "step = one call for every electron of every walker",
               roofline=roofline_block("local derivatives (table gradient + MFMA products, all kernels)",
                                       byts, ms * 1e-3))
    if cpu:
        import oracle
        k = min(W, 64 if max(s.n_elec) <= 8 else 16)
        t0 = time.perf_counter()
        done = 0
        # electrons one at a time (each one is a full pass of row-replaced
        # LUs over every determinant) until about 8 s of host time
        while time.perf_counter() - t0 < 8.0:
            oracle.grad_lap(s, wl.walkers.pos[:k], done % n_tot)
            done += 1
        dt = time.perf_counter() - t0
        row["cpu_baseline"] = dict(value=k * s.n_det * done / dt, unit="walker.det.electron/s",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"{k} walkers x {done} electrons (row-replaced full LUs, "
                                          f"{dt:.1f} s)")
    return row


def _uneven_one(j, n_moves):
    return synth_mod().uneven_instances(W=256, n_moves=n_moves, only=[j])[0]


def uneven_workloads(n_moves=4, workers=16):
    """The 64 uneven instances, generated in a process pool (the generator is
    pure Python per determinant); call before the GPU is touched."""
    import concurrent.futures as cf
    import multiprocessing as mp
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(workers, os.cpu_count() or 1),
                                mp_context=mp.get_context("fork")) as ex:
        wls = list(ex.map(_uneven_one, range(64), [n_moves] * 64))
    log(f"uneven: 64 instances generated in {time.perf_counter() - t0:.1f} s")
    return wls


def run_uneven(steps, warmup, n_moves=4, precision="fp64", wls=None, cpu=True):
    """64 instances of uneven size (n = 5..64 electrons per spin, m = 4n,
    100..200 000 determinants, 256 walkers each) moved together: one step =
    a proposal + commit of one electron in every instance, issued as one
    group launch per walker-tile size (FP64, or the mixed form)."""
    import torch
    if wls is None:
        wls = uneven_workloads(n_moves)
    # a side stream: the legacy default stream cannot be captured
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        return _run_uneven(steps, warmup, n_moves, precision, wls, cpu, stream)


def _run_uneven(steps, warmup, n_moves, precision, wls, cpu, side_stream):
    import torch
    from paper_1106_2456_amd import Context, Group
    ctxs = []
    for w in wls:
        sy = w.system
        mo = max(int(sy.exc[0].orders().max()), int(sy.exc[1].orders().max()), 1)
        c = Context(sy.n_elec, sy.n_orb, 256, max_order=mo, precision=precision, stream=side_stream)
        c.set_expansion(sy.exc[0], sy.exc[1], sy.coef, sy.det_up, sy.det_dn)
        for sp in (0, 1):
            c.set_basis(sp, sy.centres, sy.expo, sy.mo_spin(sp))
        ctxs.append(c)
    # one group: each instance keeps the walker tile its tables fit, and the
    # library runs one determinant launch per tile class inside each call
    group = Group(ctxs, [256] * len(wls), common_tile=False)
    groups = [(group, list(range(len(ctxs))))]
    moves = []
    for c, w in zip(ctxs, wls):
        pos = torch.as_tensor(w.walkers.pos, device="cuda")
        nu = w.system.n_elec[0]
        c.init(c.sgauss_eval(0, pos[:, :nu].contiguous()), c.sgauss_eval(1, pos[:, nu:].contiguous()))
    for k in range(n_moves):
        es, news, masks = [], [], []
        for c, w in zip(ctxs, wls):
            e = int(w.moves.electron[k])
            r = torch.as_tensor(w.walkers.pos[:, e] + w.moves.disp[k], device="cuda")
            es.append(e)
            news.append(c.sgauss_eval(c.spin_of(e), r.contiguous()))
            masks.append(torch.as_tensor(w.moves.accept_half[k], dtype=torch.uint8, device="cuda"))
        moves.append((es, news, masks))
    outs = [(torch.empty(256, dtype=torch.float64, device="cuda"),
             torch.empty((256, 3), dtype=torch.float64, device="cuda"),
             torch.empty(256, dtype=torch.float64, device="cuda"),
             torch.zeros(256, dtype=torch.int32, device="cuda")) for _ in wls]
    stream = group.stream
    torch.cuda.synchronize()
    # autotuned launch plans (per walker-tile class), then the state again
    group.tune(moves[0][0], moves[0][1])
    for c, w in zip(ctxs, wls):
        pos = torch.as_tensor(w.walkers.pos, device="cuda")
        nu = w.system.n_elec[0]
        c.init(c.sgauss_eval(0, pos[:, :nu].contiguous()), c.sgauss_eval(1, pos[:, nu:].contiguous()))

    def step(k):
        es, news, masks = moves[k % n_moves]
        group.propose(es, news, outs)
        group.accept(es, masks)

    for k in range(max(warmup, 1)):
        step(k)
    torch.cuda.synchronize()
    # the timed steps captured into one HIP graph, replayed once
    with group.capture() as cap:
        for k in range(steps):
            step(k)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    cap.graph.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    wdets = sum(256 * w.system.n_det for w in wls)
    st = torch.stack([o[3] for o in outs]).cpu().numpy()
    # algorithmic bytes of one step's determinant launches (every instance's
    # moving spin; the average over the timed moves)
    byts = []
    for k in range(n_moves):
        tot = 0.0
        for w in wls:
            e = int(w.moves.electron[k])
            sp = 0 if e < w.system.n_elec[0] else 1
            n, m = w.system.n_elec[sp], w.system.n_orb[sp] - w.system.n_elec[sp]
            tot += bytes_per_launch(w.system.exc[sp], 256, n, m, precision, fused=False)
        byts.append(tot)
    out = dict(value=wdets / (ms * 1e-3), unit="walker.det/s", ms_per_step=ms,
               walker_dets_per_step=wdets, status_bits=int(np.bitwise_or.reduce(st.ravel())),
               tiles={str(t): sum(1 for c in ctxs if c.get_plan(0)["walker_tile"] == t)
                      for t in sorted({c.get_plan(0)["walker_tile"] for c in ctxs})},
               workload="64 uneven instances x 256 walkers (n 5..64 per spin, m = 4n, "
                        f"N_det 1e2..2e5 log-uniform), {precision}; step = one proposal + "
                        "commit of every instance: one group call (a determinant launch per "
                        "walker-tile class), autotuned, the timed steps replayed as one HIP graph",
               roofline=roofline_block("group step (all kernels of one proposal + commit)",
                                       float(np.mean(byts)), ms * 1e-3,
                                       note="bytes: the determinant launches' algorithmic bytes "
                                            "of every instance; time: the whole step"))
    if cpu:
        out["cpu_baseline"] = uneven_cpu_baseline(wls)
    return out


def uneven_cpu_baseline(wls, n_inst=16):
    """The oracle on 2 walkers x 1 move of the n_inst instances with the
    fewest walker.det (the largest ones take minutes per walker)."""
    import oracle
    order = np.argsort([w.system.n_det * w.meta["n"] ** 3 for w in wls])
    t0 = time.perf_counter()
    wd = 0
    done = 0
    # instances in order of increasing work, 16 walkers x 1 move each, until
    # about 8 s of host time
    for i in order:
        w = wls[i]
        e = int(w.moves.electron[0])
        pos = w.walkers.pos[:16].copy()
        oracle.move(w.system, pos, e, pos[:, e] + w.moves.disp[0, :16])
        wd += 16 * w.system.n_det
        done += 1
        if time.perf_counter() - t0 > 8.0:
            break
    dt = time.perf_counter() - t0
    return dict(value=wd / dt, unit="walker.det/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"16 walkers x 1 move of the {done} instances with the least work "
                       f"(full-LU oracle, {dt:.1f} s)")


def synth_mod():
    import synth
    return synth


ALL_ROWS = ("cfg3_fp64,cfg3_mixed,cfg3_mixed_gemm,cfg4_adjoint,cfg5_uneven_fp64,cfg5_uneven_mixed,"
            "local_cfg2,local_cfg3")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="fp64,mixed,mixed_gemm")
    ap.add_argument("--walkers", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--repeat", type=int, default=8,
                    help="back-to-back determinant-kernel launches per HIP event pair")
    ap.add_argument("--rows", default=ALL_ROWS,
                    help="other rows of the path to measure (comma list of " + ALL_ROWS +
                         ", cfg3_mixed_gemm_ksum64; empty for none); reported under 'rows'")
    ap.add_argument("--row-steps", type=int, default=3,
                    help="timed sweeps of the molecular-shaped rows (64 moves each)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the forms, run a plain device copy (torch.neg, out=) of this many "
                         "MiB three times: the known-size reference for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the walkers are "
              "independent, so a multi-GPU run would shard them with no per-move "
              "communication; bench.py measures the one-GPU share.", file=sys.stderr)
        sys.exit(2)
    rows_wanted = [x for x in args.rows.split(",") if x]
    for r in rows_wanted:
        if r not in ALL_ROWS.split(",") + ["cfg3_mixed_gemm_ksum64"]:
            raise SystemExit(f"unknown row {r!r}")
    # the uneven instances are generated on the host cores before any GPU work
    uneven_wls = uneven_workloads() if any(r.startswith("cfg5") for r in rows_wanted) else None
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    import synth
    import paper_1106_2456_amd  # noqa: F401  (fails loudly without libmde.so)

    wl = synth.water_like(2, W=args.walkers)
    log(f"workload: W={wl.walkers.W} n_det={wl.system.n_det} U={wl.meta['n_exc_up']}/{wl.meta['n_exc_dn']}")
    forms = {}
    for f in [x for x in args.forms.split(",") if x]:
        r = run_form(wl, f, args.steps, args.warmup, autotune=not args.no_autotune, repeat=args.repeat)
        log(f"{f}: {r['ms_per_step']:.3f} ms/sweep  {r['value']:.3e} walker.det/s  "
            f"det kernel {r['det_avg_us']:.1f} us ({r['det_gbs']:.0f} GB/s, {r['det_tflops']:.2f} TFLOP/s; "
            f"{r['det_single_us']:.1f} us one launch per event pair) plan {r['plan'][0]}")
        forms[f] = r
    cpu = None if args.no_cpu else cpu_baseline(wl)
    rows = {}
    mol = mol_cpu = None
    for r in rows_wanted:
        t0 = time.perf_counter()
        log(f"{r}: starting")
        if r.startswith("cfg3_"):
            if mol is None:
                mol = molecular_workload()
            prec = r[len("cfg3_"):]
            rows[r] = run_molecular(*mol, prec, args.row_steps, 1)
            if not args.no_cpu:
                if mol_cpu is None:
                    mol_cpu = cpu_baseline(mol[0], probe=128, max_moves=1)
                rows[r]["cpu_baseline"] = mol_cpu
            torch.cuda.empty_cache()
        elif r == "local_cfg2":
            rows[r] = run_local(wl, args.steps, cpu=not args.no_cpu)
        elif r == "local_cfg3":
            if mol is None:
                mol = molecular_workload()
            rows[r] = run_local(mol[0], 5, cpu=not args.no_cpu, tag="molecular-shaped")
            torch.cuda.empty_cache()
        elif r == "cfg4_adjoint":
            rows[r] = run_adjoint(args.steps, args.warmup, cpu=not args.no_cpu)
        elif r.startswith("cfg5_uneven_"):
            prec = r[len("cfg5_uneven_"):]
            rows[r] = run_uneven(min(args.steps, 10), args.warmup, precision=prec, wls=uneven_wls,
                                 cpu=not args.no_cpu and r == "cfg5_uneven_fp64")
            if not args.no_cpu and r != "cfg5_uneven_fp64" and "cfg5_uneven_fp64" in rows:
                rows[r]["cpu_baseline"] = rows["cfg5_uneven_fp64"]["cpu_baseline"]
            torch.cuda.empty_cache()
        rf = rows[r].get("roofline", {})
        log(f"{r}: {rows[r]['ms_per_step']:.3f} ms/step  {rows[r]['value']:.3e} walker.det/s  "
            f"roofline {rf.get('frac', float('nan')):.3f} of HBM ({time.perf_counter() - t0:.0f} s)")
    if args.copy_mib > 0:
        x = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        log(f"copy reference: 3 x torch.neg over {args.copy_mib} MiB (read + write each)")
        del x, y
    if not forms:
        # rows only (e.g. `--forms "" --rows cfg4_adjoint` under a profiler)
        print(json.dumps({"rows": rows}))
        return
    head = forms.get("fp64") or next(iter(forms.values()))
    achieved = head["det_gbs"]
    traffic = measured_traffic(head["plan"]) if head["precision"] == "fp64" else None
    out = {
        "metric": "excited-det ratios/s (walker.det, +grad/lap) mixed/batched vs plain FP64",
        "value": head["value"],
        "unit": "walker.det/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head["precision"] == "fp64" else "f32-table/f64",
        "data": "synthetic (seeded s-Gaussian water-like system)",
        "config": {"workload": "water-like batched: 5+5 electrons, 5+20 orbitals/spin, "
                               "10000 determinants (orders 1-4), 4096 walkers, FP64; "
                               "step = one sweep of 10 single-electron moves, 50% accepted",
                   "walkers": wl.walkers.W, "n_det": wl.system.n_det,
                   "moves_per_step": sum(wl.system.n_elec), "precision": head["precision"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE)",
                     "kernel": "k_det<double, propose>",
                     "launch_us": head["det_avg_us"],
                     "launch_us_one_per_event_pair": head["det_single_us"],
                     "launches_per_event_pair": head["det_repeat"],
                     "bytes_per_launch": head["det_bytes_per_launch"],
                     "alu": {"achieved": head["det_tflops"], "peak": PEAK_FP64_VECTOR_TFLOPS,
                             "unit": "TFLOP/s", "frac": head["det_tflops"] / PEAK_FP64_VECTOR_TFLOPS,
                             "flops_per_launch": head["det_flops_per_launch"]}},
        "cpu_baseline": cpu,
        "forms": {k: {kk: v[kk] for kk in ("value", "ms_per_step", "ms_per_step_eager", "det_avg_us",
                                           "det_single_us", "det_gbs", "det_tflops", "status_bits",
                                           "plan")}
                  for k, v in forms.items()},
    }
    if rows:
        out["rows"] = rows
    print(json.dumps(out))


if __name__ == "__main__":
    main()
