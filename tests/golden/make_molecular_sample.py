"""Expected values of the molecular-shaped full-size parity sample, written
by the CPU oracle alone (no GPU code is imported):

    python tests/golden/make_molecular_sample.py

Workload: n = 32 electrons per spin, 32 occupied + 224 virtual orbitals per
spin from 512 s-Gaussians on 20 nuclei in a 12 bohr box, 100 000
determinants of orders 1-4, 2 048 walkers (the molecular-shaped mixed-
precision workload).  Sample: walkers 0, 64, .., 1984 (one per 64-walker
tile, every position in a smaller tile), 10 moves alternating the two spins
(a spin change at every move), seeded 50 % acceptance.  Stored per move and
sampled walker: ratio, grad, lap, their condition-aware scales, and the
first-order FP32-entry scales (tables kept in FP32 across commits, with
their propagated entry errors; product-formed entries).

The inputs whose generation goes through a math library (the MO matrix from
a QR factorisation, exponents and CI coefficients through exp) can differ
in the last bit between machines, so the file stores them and ``load``
puts them into the regenerated workload; a fingerprint of the remaining
inputs guards against generator drift.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "molecular_n32_sample.npz")
ELECTRONS = [0, 32, 5, 40, 11, 47, 20, 58, 31, 63]
SAMPLE = np.arange(0, 2048, 64)


def workload():
    return synth.molecular(3, W=2048, n_det=100000, n_moves=len(ELECTRONS),
                           electron_order=ELECTRONS)


def fingerprint(wl) -> str:
    s = wl.system
    h = hashlib.sha256()
    for a in (wl.walkers.pos, wl.moves.disp, wl.moves.accept_half, s.det_up, s.det_dn,
              s.exc[0].offsets, s.exc[0].holes, s.exc[0].particles, s.exc[1].offsets,
              s.exc[1].holes, s.exc[1].particles, s.centres):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:32]


N_ORB = 256   # orbitals per spin: MO rows used


def load():
    """(workload with the stored inputs, stored data)"""
    g = np.load(OUT, allow_pickle=False)
    wl = workload()
    s = wl.system
    s.mo = np.ascontiguousarray(g["in_mo"])
    s.expo = np.ascontiguousarray(g["in_expo"])
    s.coef = np.ascontiguousarray(g["in_coef"])
    return wl, g


def main():
    t0 = time.time()
    wl = workload()
    s = wl.system
    print(f"generated in {time.time() - t0:.1f} s; U = {s.exc[0].n_exc}/{s.exc[1].n_exc}",
          flush=True)
    s.mo = np.ascontiguousarray(s.mo[:N_ORB])
    pos = wl.walkers.pos[SAMPLE].copy()
    rec = {k: [] for k in ("ratio", "grad", "lap", "sc_ratio", "sc_grad", "sc_lap",
                           "x_round", "x_gemm")}
    # no from-scratch refresh happens within the 10 moves (once per 64 commits)
    track = oracle.StoredTableErrors(s, pos)
    for k, e in enumerate(ELECTRONS):
        new_r = pos[:, e] + wl.moves.disp[k, SAMPLE]
        r = oracle.move(s, pos, e, new_r)
        m = track.scales(pos, e, new_r)
        rec["ratio"].append(r["ratio"])
        rec["grad"].append(r["grad"])
        rec["lap"].append(r["lap"])
        rec["sc_ratio"].append(r["scale_ratio"])
        rec["sc_grad"].append(r["scale_grad"])
        rec["sc_lap"].append(r["scale_lap"])
        rec["x_round"].append(m["round"])
        rec["x_gemm"].append(m["gemm"])
        acc = wl.moves.accept_half[k, SAMPLE].astype(bool)
        track.commit(acc)
        pos[acc, e] = new_r[acc]
        print(f"move {k} (electron {e}) done at {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, sample=SAMPLE, electrons=np.asarray(ELECTRONS),
                        fingerprint=np.asarray(fingerprint(wl)), in_mo=s.mo, in_expo=s.expo,
                        in_coef=s.coef, **{k: np.asarray(v) for k, v in rec.items()})
    print("wrote", OUT)


if __name__ == "__main__":
    main()
