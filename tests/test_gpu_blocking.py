"""Blocking and work-split knobs change only the order of FP64 sums: every
setting must reproduce the oracle, and the settings agree with each other to
FP64 rounding.

* Cholesky / inverse outer block (CPM_CHOL_BLOCK): 64 (one level), 256
  (default), 1024, on the 2880-atom capacitor (2880 = 11.25 blocks of 256: a
  ragged last block) against the stored oracle rows of S.
* Real-space charge order (CPM_RS_SORT_MIN): z-ordered blocks with skipping
  against the caller's order, small capacitor, 20 snapshots.
* CG vector grid (CPM_CG_BLOCKS): one workgroup against the default.
"""
import os
import sys

import numpy as np
import pytest

from oracle import cpm_oracle as O
from paper_2203_15461_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "graphite_capacitor_2880.npz")


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


def test_cholesky_block_sizes(cpm, monkeypatch):
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    golden = dict(np.load(GOLDEN))
    w = I.graphite_capacitor()
    rows = golden["rows"]
    Ss = {}
    for ob in (64, 256, 1024):
        monkeypatch.setenv("CPM_CHOL_BLOCK", str(ob))
        say(f"graphite_capacitor_2880: Cholesky outer block {ob}")
        ctx = cpm.setup(w)
        S = ctx.copy_matrix(2, torch.empty((w.n, w.n), dtype=torch.float64, device="cuda"))
        u = ctx.copy_vector(0, torch.empty(w.n, dtype=torch.float64, device="cuda"))
        ctx.synchronize()
        Ss[ob] = S.cpu().numpy()
        ctx.close()
        assert rel(Ss[ob][rows], golden["S_rows"]) < 1e-10
        assert rel(u.cpu().numpy(), golden["u"]) < 1e-10
    assert rel(Ss[64], Ss[256]) < 1e-12
    assert rel(Ss[1024], Ss[256]) < 1e-12


def _b(C, w, xyz):
    ctx = C.setup(w)
    x = torch.as_tensor(np.stack(xyz), dtype=torch.float64, device="cuda").contiguous()
    b = torch.empty((len(xyz), w.n), dtype=torch.float64, device="cuda")
    ctx.potential_vector(x, b)
    ctx.synchronize()
    ctx.close()
    return b.cpu().numpy()


def test_charge_order_of_real_space(cpm, monkeypatch):
    w = I.small_capacitor("a")
    xyz = [I.snapshot(w, s) for s in range(20)]
    say("real space: z-ordered charges vs caller order, 20 snapshots")
    monkeypatch.setenv("CPM_RS_SORT_MIN", "1")
    b_sorted = _b(cpm, w, xyz)
    monkeypatch.setenv("CPM_RS_SORT_MIN", "1000000000")
    b_plain = _b(cpm, w, xyz)
    p = O.params_for(w)
    ref = np.array([O.potential_vector(w.electrode_xyz, r, w.electrolyte_q, p) for r in xyz[:3]])
    assert rel(b_sorted[:3], ref) < 1e-10
    assert rel(b_plain[:3], ref) < 1e-10
    assert rel(b_sorted, b_plain) < 1e-13


def test_cg_grid_sizes(cpm, monkeypatch):
    w = I.small_capacitor("b")
    xyz = torch.as_tensor(np.stack([I.snapshot(w, s) for s in range(3)]), dtype=torch.float64,
                          device="cuda").contiguous()
    qs = []
    for cap in ("1", None):
        if cap is None:
            monkeypatch.delenv("CPM_CG_BLOCKS", raising=False)
        else:
            monkeypatch.setenv("CPM_CG_BLOCKS", cap)
        say(f"CG vector grid cap {cap or 'default'}")
        ctx = cpm.setup(w, matrix_free=True)
        b = torch.empty((3, w.n), dtype=torch.float64, device="cuda")
        ctx.potential_vector(xyz, b)
        q = torch.empty_like(b)
        ctx.solve_cg(b, q, tol=1e-13)
        ctx.synchronize()
        qs.append(q.cpu().numpy())
        ctx.close()
    assert rel(qs[0], qs[1]) < 1e-11
    assert np.all(np.abs(qs[0].sum(1)) <= 1e-12)


def test_z_order_with_fewer_charges_than_a_block(cpm):
    """Two ions, a batch of 20 (z-ordered path): one partial 64-charge block,
    so most real-space chunks are empty and must contribute zero."""
    w = I.small_capacitor("b", n_ions=2)
    xyz = [I.snapshot(w, s) for s in range(20)]
    say(f"z-ordered real space with m = {w.m}, batch 20")
    b = _b(cpm, w, xyz)
    p = O.params_for(w)
    ref = np.array([O.potential_vector(w.electrode_xyz, r, w.electrolyte_q, p) for r in xyz[:4]])
    assert rel(b[:4], ref) < 1e-10


def test_assembly_deferred_to_first_consumer(cpm):
    """cpm_build_elastance leaves the assembly of A to its first consumer:
    cpm_copy_matrix(0) and cpm_apply_elastance without any cpm_invert, and
    an asynchronous cpm_invert, all see the same A (the oracle's)."""
    w = I.small_capacitor("a")
    p = O.params_for(w)
    A_ref = O.elastance(w.electrode_xyz, p)
    R = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device="cuda").contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device="cuda").contiguous()
    say("deferred assembly: copy, apply, asynchronous inversion")
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    ctx.build_elastance(R, eid, 2)
    A = ctx.copy_matrix(0, torch.empty((w.n, w.n), dtype=torch.float64, device="cuda"))
    ctx.synchronize()
    assert rel(A.cpu().numpy(), A_ref) < 1e-11
    ctx.build_elastance(R, eid, 2)                     # pending again: apply assembles it
    x = torch.as_tensor(np.random.default_rng(5).normal(size=(3, w.n)), device="cuda").contiguous()
    y = torch.empty_like(x)
    ctx.apply_elastance(x, y)
    ctx.synchronize()
    assert rel(y.cpu().numpy(), x.cpu().numpy() @ A_ref.T) < 1e-11
    ctx.build_elastance(R, eid, 2)
    ctx.invert(cpm.STORE_F64 | cpm.INVERT_ASYNC)       # assembly on the second stream
    S = ctx.copy_matrix(2, torch.empty((w.n, w.n), dtype=torch.float64, device="cuda"))
    A2 = ctx.copy_matrix(0, torch.empty((w.n, w.n), dtype=torch.float64, device="cuda"))
    ctx.synchronize()
    assert rel(A2.cpu().numpy(), A_ref) < 1e-11
    assert rel(S.cpu().numpy(), O.capacitance(A_ref).S) < 1e-10
    ctx.close()
