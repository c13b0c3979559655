#!/usr/bin/env python3
"""Throughput of the multi-determinant table method on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp64,mixed]

Workload (headline): the water-like batched system -- 5 up + 5 down
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
precision forms.  `--rows adjoint,uneven` adds two more rows of the path
under "rows": the adjoint (forward from the tables + backward, 1024 walkers,
FP64, with the oracle timed beside it) and 64 uneven instances moved
together, one group launch per walker-tile size.
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
# accumulations); FMA counts 2.  See the design doc for the derivation.
DET_FLOPS = {1: 26, 2: 43, 3: 80, 4: 165}


def det_flops(k: int) -> int:
    if k in DET_FLOPS:
        return DET_FLOPS[k]
    # generic path: k+1 eliminations of k x k (2k^3/3 each) + 4(2k+2) + 10
    return int((k + 1) * 2 * k ** 3 / 3 + 4 * (2 * k + 2) + 10)


def flops_per_launch(exc, W: int) -> float:
    orders = exc.orders()
    return float(W) * sum(det_flops(int(k)) for k in orders if k > 0)


def bytes_per_launch(exc, W: int, n: int, m: int, precision: str) -> float:
    """Algorithmic HBM bytes of one determinant-kernel launch: each walker's CI
    weight C_u of every excitation of the moving spin (8 B, read once), the
    walker's inputs once and its output sums once.  FP64 form (the kernel
    forms the proposal itself): T [n*m], the inverse [n*n], the new orbital
    values and their gradient and laplacian [5(n+m)], six sums out.  Mixed
    forms: FP32 T' [n*m], g^a [4m], c' [n], five sums out."""
    U = int((exc.orders() > 0).sum())
    if precision == "fp64":
        return float(W) * (8 * U + 8 * (n * m + n * n + 5 * (n + m)) + 6 * 8)
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


def run_form(wl, precision, steps, warmup, autotune=True, repeat=8):
    """Time `steps` sweeps (one graph) of one precision form; returns a dict."""
    import torch
    s = wl.system
    W = wl.walkers.W
    n_tot = s.n_elec[0] + s.n_elec[1]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = build_context(wl, precision, stream, refresh_every=n_tot)
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
    by = np.mean([bytes_per_launch(s.exc[sp], W, s.n_elec[sp], s.n_orb[sp] - s.n_elec[sp], precision)
                  for sp in (ctx.spin_of(m[0]) for m in moves)])
    det_avg_s = det_ms / max(det_n, 1) / 1e3
    return dict(precision=precision, ms_per_step=ms_step, value=wdets / (ms_step / 1e3),
                ms_per_step_eager=ms_eager / steps,
                det_launches=det_n, det_avg_us=det_avg_s * 1e6, det_flops_per_launch=fl,
                det_single_us=single_ms / max(single_n, 1) * 1e3, det_repeat=repeat,
                det_bytes_per_launch=by,
                det_gbs=by / det_avg_s / 1e9 if det_n else None,
                det_tflops=fl / det_avg_s / 1e12 if det_n else None, plan=plan,
                status_bits=int(np.bitwise_or.reduce(st.ravel())) if st.size else 0)


def cpu_baseline(wl, target_seconds=12.0):
    """The oracle on a bounded sample of the same workload (the first walkers,
    the first moves of the sweep), on the host cores."""
    import oracle
    s = wl.system
    threads = oracle.num_threads()
    n_tot = sum(s.n_elec)
    # size the walker sample so that one sweep takes about target_seconds
    probe = min(wl.walkers.W, 64)
    t0 = time.perf_counter()
    e = int(wl.moves.electron[0])
    oracle.move(s, wl.walkers.pos[:probe].copy(), e, wl.walkers.pos[:probe, e] + wl.moves.disp[0, :probe])
    per_walker_move = (time.perf_counter() - t0) / probe
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
    out = dict(value=W * s.n_det / (ms * 1e-3), unit="walker.det/s", ms_per_step=ms,
               workload=f"water-like, {W} walkers, {s.n_det} determinants, FP64; "
                        "step = forward from the tables + backward (grad_c, grad_T)")
    if cpu:
        import oracle
        k = min(W, 256)
        tu, td = Tu[:k].cpu().numpy(), Td[:k].cpu().numpy()
        t0 = time.perf_counter()
        oracle.tables(s, tu, td)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=k * s.n_det / dt, unit="walker.det/s",
                                   cores=oracle.num_threads(), kind="oracle",
                                   sample=f"{k} walkers, forward + adjoint by full LU ({dt:.2f} s)")
    return out


def run_uneven(steps, warmup, n_moves=4, precision="fp64"):
    """64 instances of uneven size (n = 5..64 electrons per spin, m = 4n,
    100..200 000 determinants, 256 walkers each) moved together: one step =
    a proposal + commit of one electron in every instance, issued as one
    group launch per walker-tile size (FP64, or the mixed form)."""
    import torch
    from paper_1106_2456_amd import Context, Group
    log("uneven: generating 64 instances")
    wls = synth_mod().uneven_instances(W=256, n_moves=n_moves)
    ctxs = []
    for w in wls:
        sy = w.system
        mo = max(int(sy.exc[0].orders().max()), int(sy.exc[1].orders().max()), 1)
        c = Context(sy.n_elec, sy.n_orb, 256, max_order=mo, precision=precision)
        c.set_expansion(sy.exc[0], sy.exc[1], sy.coef, sy.det_up, sy.det_dn)
        for sp in (0, 1):
            c.set_basis(sp, sy.centres, sy.expo, sy.mo_spin(sp))
        ctxs.append(c)
    # one group launch per walker-tile size (the instances whose tables fit
    # wide tiles keep them)
    groups = Group.by_tile(ctxs, [256] * len(wls))
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
    stream = groups[0][0].stream
    torch.cuda.synchronize()

    def step(k):
        es, news, masks = moves[k % n_moves]
        for g, idx in groups:
            g.propose([es[i] for i in idx], [news[i] for i in idx], [outs[i] for i in idx])
            g.accept([es[i] for i in idx], [masks[i] for i in idx])

    for k in range(max(warmup, 1)):
        step(k)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        step(k)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    wdets = sum(256 * w.system.n_det for w in wls)
    st = torch.stack([o[3] for o in outs]).cpu().numpy()
    return dict(value=wdets / (ms * 1e-3), unit="walker.det/s", ms_per_step=ms,
                walker_dets_per_step=wdets, status_bits=int(np.bitwise_or.reduce(st.ravel())),
                tiles={str(ctxs[idx[0]].get_plan(0)["walker_tile"]): len(idx) for _, idx in groups},
                workload="64 uneven instances x 256 walkers (n 5..64 per spin, m = 4n, "
                         f"N_det 1e2..2e5 log-uniform), {precision}; step = one proposal + "
                         "commit of every instance, one group launch per walker-tile size, eager")


def synth_mod():
    import synth
    return synth


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
    ap.add_argument("--rows", default="",
                    help="also measure these other rows of the path (comma list of "
                         "adjoint, uneven, uneven_mixed); reported under 'rows'")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the forms, run a plain device copy (torch.neg, out=) of this many "
                         "MiB three times: the known-size reference for the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the walkers are "
              "independent, so a multi-GPU run would shard them with no per-move "
              "communication; this build measures the one-GPU share.", file=sys.stderr)
        sys.exit(2)
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
    rows = {}
    for r in [x for x in args.rows.split(",") if x]:
        if r == "adjoint":
            rows[r] = run_adjoint(args.steps, args.warmup, cpu=not args.no_cpu)
        elif r == "uneven":
            rows[r] = run_uneven(min(args.steps, 10), args.warmup)
        elif r == "uneven_mixed":
            rows[r] = run_uneven(min(args.steps, 10), args.warmup, precision="mixed")
        else:
            raise SystemExit(f"unknown row {r!r}")
        log(f"{r}: {rows[r]['ms_per_step']:.3f} ms/step  {rows[r]['value']:.3e} walker.det/s")
    if args.copy_mib > 0:
        x = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.neg(x, out=y)
        torch.cuda.synchronize()
        log(f"copy reference: 3 x torch.neg over {args.copy_mib} MiB (read + write each)")
        del x, y
    if not forms:
        # rows only (e.g. `--forms "" --rows adjoint` under a profiler)
        print(json.dumps({"rows": rows}))
        return
    head = forms.get("fp64") or next(iter(forms.values()))
    cpu = None if args.no_cpu else cpu_baseline(wl)
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
