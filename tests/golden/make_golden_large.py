"""Write the stored oracle results for the large-system GPU parity tests.

    python tests/golden/make_golden_large.py [--alpha A ...] [--jobs J]

Calls only the seeded input generator and the FP64 oracle (oracle/).

* Scaled graphite capacitors (scaled_graphite_capacitor(target); by default
  the 20064-atom one: 2 x 3 AB layers of 3344 atoms, 93.7 x 93.5 A, 50 A
  gap, 10 water charges per electrode atom + 1 M ions, m = 201168; also the
  8400-atom one of the CG tests): for each Ewald alpha asked for
  (r_c = 3.6 / alpha, so erfc(alpha r_c) stays that of alpha 0.3, r_c 12 A;
  k-space accuracy 1e-8), sampled rows of A and of b with the full
  electrolyte (snapshots 0, 1 at 20064 atoms; 0-2 at 8400).  The oracle cannot invert A at this size in a
  test's time, so charges are checked through these rows: A_rows q - b_rows
  - v_rows must be one uniform value mu on every row (the Lagrange
  multiplier of e^T q = 0).
* The smallest capacitor of the uneven eight-capacitor batch (targets drawn
  with seed 5 from U{2000..20000}): the full oracle run, A, S, b, q and the
  electrode totals for snapshots 0-2, at alpha 0.3, r_c 12 A.

The structure factor of 2e5 charges over 1e5-2.4e5 k-vectors takes the
oracle tens of minutes per snapshot; the (alpha, snapshot) tasks run in
parallel processes.
"""
import argparse
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cpm_oracle as O  # noqa: E402
from paper_2203_15461_amd import inputs as I  # noqa: E402

SNAPS_ROWS = {20000: (0, 1), 8500: (0, 1, 2)}
SNAPS_C5 = (0, 1, 2)


def input_hash(w, snaps) -> str:
    h = hashlib.sha256()
    for a in (w.electrode_xyz, w.electrode_id.astype(np.int64), w.electrolyte_q, *snaps):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def large_params(w, alpha):
    return O.params_for(w, alpha=alpha, rcut=3.6 / alpha)


def sample_rows(w):
    """Two rows at each boundary between electrode planes, first and last."""
    per = w.n // 6
    return np.array(sorted({0, 1, w.n - 2, w.n - 1} |
                           {k * per + d for k in range(1, 6) for d in (-1, 0)}))


def task_b_rows(args):
    target, alpha, s = args
    w = I.scaled_graphite_capacitor(target)
    p = large_params(w, alpha)
    return (target, alpha, s, O.potential_vector(w.electrode_xyz, I.snapshot(w, s),
                                                 w.electrolyte_q, p, rows=sample_rows(w)))


def task_a_rows(args):
    target, alpha = args
    w = I.scaled_graphite_capacitor(target)
    return (target, alpha), O.elastance(w.electrode_xyz, large_params(w, alpha), rows=sample_rows(w))


def c5_targets():
    rng = np.random.default_rng(5)
    return sorted(int(t) for t in rng.integers(2000, 20001, size=8))


def task_c5():
    w = I.scaled_graphite_capacitor(c5_targets()[0])
    p = O.params_for(w)
    snaps = [I.snapshot(w, s) for s in SNAPS_C5]
    A = O.elastance(w.electrode_xyz, p)
    cap = O.capacitance(A)
    v = O.applied_potential(w.electrode_id, w.v_electrode)
    bs = [O.potential_vector(w.electrode_xyz, r, w.electrolyte_q, p) for r in snaps]
    qs = [O.charges(cap.S, b, v) for b in bs]
    Qs = [O.electrode_totals(q, w.electrode_id, 2) for q in qs]
    out = os.path.join(HERE, f"{w.name}.npz")
    rows = np.linspace(0, w.n - 1, 8).astype(np.int64)
    np.savez_compressed(out, rows=rows, A_rows=A[rows], S_rows=cap.S[rows], u=cap.u, s=cap.s,
                        b=np.array(bs), q=np.array(qs), Q=np.array(Qs), n=w.n, m=w.m,
                        nk=len(O.kvectors(p)[2]), snapshots=np.array(SNAPS_C5),
                        input_sha256=input_hash(w, snaps))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--alpha", type=float, nargs="*", default=[0.3])
    ap.add_argument("--targets", type=int, nargs="*", default=[20000],
                    help="scaled capacitors (electrode atom targets) to store sampled rows for")
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--skip-c5", action="store_true")
    a = ap.parse_args()
    from multiprocessing import Pool
    with Pool(a.jobs) as pool:
        c5 = None if a.skip_c5 else pool.apply_async(task_c5)
        btasks = [(t, al, s) for t in a.targets for al in a.alpha for s in SNAPS_ROWS[t]]
        brows = pool.map_async(task_b_rows, btasks)
        arows = pool.map_async(task_a_rows, [(t, al) for t in a.targets for al in a.alpha])
        bres, ares = brows.get(), dict(arows.get())
        for t in a.targets:
            w = I.scaled_graphite_capacitor(t)
            snaps = [I.snapshot(w, s) for s in SNAPS_ROWS[t]]
            rows = sample_rows(w)
            for al in a.alpha:
                p = large_params(w, al)
                b = np.array([r for (tt, x, s, r) in sorted(bres, key=lambda e: e[:3])
                              if tt == t and x == al])
                out = os.path.join(HERE, f"{w.name}_rows_alpha{al:.2f}.npz")
                np.savez_compressed(out, rows=rows, A_rows=ares[(t, al)], b_rows=b,
                                    v_rows=O.applied_potential(w.electrode_id, w.v_electrode)[rows],
                                    alpha=al, rcut=p.rcut, nk=len(O.kvectors(p)[2]),
                                    snapshots=np.array(SNAPS_ROWS[t]),
                                    input_sha256=input_hash(w, snaps))
                print("wrote", out, flush=True)
        if c5 is not None:
            print("wrote", c5.get(), flush=True)


if __name__ == "__main__":
    main()
