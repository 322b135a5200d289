"""The factor-only inverse (CPM_INVERT_FACTOR): A = L L^T kept, A^-1 x by
forward and back substitution, S (b + v) = P A^-1 b + d (Eqs. 3-6).

Checked against the stored oracle results of the 2880-atom capacitor (q and
electrode totals at 1e-10, |sum q| <= 1e-12 e), against the S path of the
same context parameters (s = e^T A^-1 e, q for an arbitrary per-atom
potential, the finite-field response), on the 20064-atom capacitor through
the stored oracle rows (the bench's factor step, alpha 0.19), and for the
calls that need S itself, which must refuse with CPM_ESTATE.
"""
import os
import sys

import numpy as np
import pytest

from paper_2203_15461_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def cpm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_15461_amd import cpm as C
    C.lib()
    return C


def _context(C, w, flags):
    ctx = C.Context(C.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    xyz = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device="cuda").contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device="cuda").contiguous()
    ctx.build_elastance(xyz, eid, int(w.electrode_id.max()) + 1)
    ctx.invert(flags)
    ctx.set_potential(w.v_electrode)
    return ctx


def test_factor_solve_2880_against_oracle(cpm):
    g = np.load(os.path.join(GOLDEN, "graphite_capacitor_2880.npz"))
    w = I.graphite_capacitor()
    say("2880 atoms, factor-only inverse, FP64 b, three oracle snapshots")
    ctx = _context(cpm, w, cpm.STORE_F64 | cpm.INVERT_FACTOR)
    xyz = torch.as_tensor(np.stack([I.snapshot(w, int(s)) for s in g["snapshots"]]),
                          dtype=torch.float64, device="cuda").contiguous()
    b = torch.empty((xyz.shape[0], w.n), dtype=torch.float64, device="cuda")
    q = torch.empty_like(b)
    Qe = torch.empty((xyz.shape[0], 2), dtype=torch.float64, device="cuda")
    ctx.potential_vector(xyz, b)
    ctx.solve_charges(b, 0x000, q, Qe)
    torch.cuda.synchronize()
    eq, eQ = rel(q.cpu().numpy(), g["q"]), rel(Qe.cpu().numpy(), g["Q"])
    say(f"  q vs oracle {eq:.3e}, Q {eQ:.3e}, |sum q| {float(q.sum(1).abs().max()):.1e}")
    assert eq < 1e-10 and eQ < 1e-10
    assert float(q.sum(1).abs().max()) <= 1e-12
    ctx.close()


def test_factor_matches_S_path(cpm):
    """s, q for the electrode potentials and for an arbitrary per-atom
    potential, from the factor and from S, on one 2880-atom configuration
    set (FP64 both ways)."""
    w = I.graphite_capacitor()
    xyz = torch.as_tensor(np.stack([I.snapshot(w, k) for k in range(70)]), dtype=torch.float64,
                          device="cuda").contiguous()
    out = {}
    rng = np.random.default_rng(11)
    v_atoms = rng.uniform(-1.0, 1.0, w.n)
    for name, flags in (("S", cpm.STORE_F64), ("factor", cpm.STORE_F64 | cpm.INVERT_FACTOR)):
        ctx = _context(cpm, w, flags)
        b = torch.empty((70, w.n), dtype=torch.float64, device="cuda")
        q = torch.empty_like(b)
        ctx.potential_vector(xyz, b)
        ctx.solve_charges(b, 0x000, q)
        ctx.set_potential_atoms(v_atoms)
        q2 = torch.empty_like(b)
        ctx.solve_charges(b[:3], 0x000, q2[:3])
        torch.cuda.synchronize()
        out[name] = (ctx.info("s_sum"), q.cpu().numpy(), q2[:3].cpu().numpy())
        ctx.close()
    es = abs(out["S"][0] - out["factor"][0]) / abs(out["S"][0])
    e1, e2 = rel(out["factor"][1], out["S"][1]), rel(out["factor"][2], out["S"][2])
    say(f"  s: {es:.2e}; q (70 configurations, batched) {e1:.2e}; q with per-atom v {e2:.2e}")
    assert es < 1e-12 and e1 < 1e-11 and e2 < 1e-11


def test_factor_async_inversion_overlaps_b(cpm):
    """The bench's step with the factor: assembly and factorisation on the
    second stream while b runs; charges equal to the synchronous ones."""
    w = I.graphite_capacitor()
    xyz = torch.as_tensor(np.stack([I.snapshot(w, k) for k in range(5)]), dtype=torch.float64,
                          device="cuda").contiguous()
    R = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device="cuda").contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device="cuda").contiguous()
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    qs = []
    for flags in (cpm.INVERT_FACTOR, cpm.INVERT_FACTOR | cpm.INVERT_ASYNC):
        ctx.build_elastance(R, eid, 2)
        ctx.invert(cpm.STORE_F64 | flags)
        b = torch.empty((5, w.n), dtype=torch.float64, device="cuda")
        ctx.potential_vector(xyz, b)
        ctx.set_potential(w.v_electrode)
        q = torch.empty_like(b)
        ctx.solve_charges(b, 0x000, q)
        torch.cuda.synchronize()
        qs.append(q.cpu().numpy())
    ctx.close()
    assert np.array_equal(qs[0], qs[1])


def test_factor_refuses_calls_that_need_S(cpm):
    w = I.graphite_capacitor()
    ctx = _context(cpm, w, cpm.STORE_F64 | cpm.INVERT_FACTOR)
    b = torch.zeros((2, w.n), dtype=torch.float64, device="cuda")
    q = torch.empty_like(b)
    out = torch.empty((w.n, w.n), dtype=torch.float64, device="cuda")
    calls = [lambda: ctx.solve_charges(b, 0x102, q),
             lambda: ctx.solve_charges(b, 0x100, q),
             lambda: ctx.set_charge([0.5, -0.5]),
             lambda: ctx.copy_matrix(2, out),
             lambda: ctx.copy_matrix(1, out)]
    for call in calls:
        with pytest.raises(cpm.CpmError) as ei:
            call()
        assert ei.value.status == cpm.ESTATE
    with pytest.raises(cpm.CpmError) as ei:
        ctx.invert(cpm.STORE_F64 | cpm.STORE_BF16X2 | cpm.INVERT_FACTOR)
    assert ei.value.status == cpm.EINVAL
    ctx.close()


def test_factor_20064_against_oracle_rows(cpm):
    """The 20064-atom capacitor (alpha 0.19, the bench's split) with the
    factor-only inverse: b rows at 1e-10 and A q - b - v uniform on every
    stored row to 1e-10."""
    path = os.path.join(GOLDEN, "scaled_graphite_capacitor_20064_rows_alpha0.19.npz")
    if not os.path.exists(path):
        pytest.skip("scaled_graphite_capacitor_20064_rows_alpha0.19.npz not generated")
    g = np.load(path)
    w = I.scaled_graphite_capacitor(20000).with_(alpha=float(g["alpha"]), rcut=float(g["rcut"]))
    say(f"20064 atoms, factor-only inverse, alpha {float(g['alpha'])}")
    ctx = _context(cpm, w, cpm.STORE_F64 | cpm.INVERT_FACTOR)
    xyz = torch.as_tensor(np.stack([I.snapshot(w, int(s)) for s in g["snapshots"]]),
                          dtype=torch.float64, device="cuda").contiguous()
    b = torch.empty((xyz.shape[0], w.n), dtype=torch.float64, device="cuda")
    q = torch.empty_like(b)
    ctx.potential_vector(xyz, b)
    ctx.solve_charges(b, 0x000, q)
    torch.cuda.synchronize()
    rows = g["rows"]
    eb = rel(b.cpu().numpy()[:, rows], g["b_rows"])
    say(f"  b rows vs oracle {eb:.3e}")
    assert eb < 1e-10
    qn = q.cpu().numpy()
    for s in range(len(g["snapshots"])):
        r = g["A_rows"] @ qn[s] - g["b_rows"][s] - g["v_rows"]
        res = float(np.abs(r - r.mean()).max() / np.abs(g["b_rows"][s] + g["v_rows"]).max())
        say(f"  snapshot {s}: non-uniform residual {res:.3e}, |sum q| {abs(qn[s].sum()):.1e}")
        assert res < 1e-10
        assert abs(qn[s].sum()) <= 1e-12
    ctx.close()
