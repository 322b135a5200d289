"""Conjugate-gradient charges (cpm_solve_cg) and the matrix-free elastance
operator (cpm_build_operator, cpm_apply_elastance) against the FP64 oracle.

The CG solve converges to q = S (b + v) (Eqs. 3-6): at tol = 1e-13 the
charges must match the oracle within 1e-10 relative (max-norm, the FP64
bar), |sum q| <= 1e-12 e, electrode totals within 1e-10.  The operator must
reproduce A x within 1e-12 relative of max |A x| for any x (the dense A
agrees with the oracle to 1e-11, so the operator is held to the oracle's A
directly).  The 2880-atom capacitor is checked against the stored oracle
rows and charges (tests/golden).
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


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dt, device="cuda").contiguous()


def _b(ctx, w, snaps, f32=False):
    xyz = _dev(np.stack([I.snapshot(w, s) for s in snaps]))
    b = torch.empty((len(snaps), w.n), dtype=torch.float32 if f32 else torch.float64, device="cuda")
    ctx.potential_vector(xyz, b)
    return b


def _oracle(w, snaps, p=None, v=None, diag=None):
    p = p or O.params_for(w)
    A = O.elastance(w.electrode_xyz, p)
    if diag is not None:
        A = A + np.diag(diag)
    S = O.capacitance(A).S
    v = O.applied_potential(w.electrode_id, w.v_electrode) if v is None else v
    bs = np.array([O.potential_vector(w.electrode_xyz, I.snapshot(w, s), w.electrolyte_q, p)
                   for s in snaps])
    qs = np.array([O.charges(S, b, v) for b in bs])
    return A, bs, qs


@pytest.mark.parametrize("variant", ["a", "b"])
def test_operator_matches_oracle_A(cpm, variant):
    """A x by the operator for random and unit vectors (all columns: x = I)."""
    w = I.small_capacitor(variant)
    say(f"operator A x small_capacitor_{variant} n={w.n}")
    ctx = cpm.setup(w, matrix_free=True)
    assert ctx.info("ell_width") > 0
    A = O.elastance(w.electrode_xyz, O.params_for(w))
    rng = np.random.default_rng(5)
    X = np.vstack([np.eye(w.n), rng.standard_normal((7, w.n))])     # n + 7 vectors: ragged groups
    Y = ctx.apply_elastance(_dev(X), torch.empty((len(X), w.n), dtype=torch.float64,
                                                 device="cuda")).cpu().numpy()
    ref = X @ A                                                          # A symmetric
    for k in range(len(X)):
        assert np.abs(Y[k] - ref[k]).max() <= 1e-12 * np.abs(ref[k]).max(), k
    ctx.close()


@pytest.mark.parametrize("matrix_free", [True, False])
def test_cg_matches_oracle(cpm, matrix_free):
    w = I.small_capacitor("a")
    snaps = list(range(35))                      # two groups: 32 + 3
    say(f"cg small_capacitor_a matrix_free={matrix_free} batch={len(snaps)}")
    ctx = cpm.setup(w, matrix_free=matrix_free)
    b = _b(ctx, w, snaps)
    q = torch.full_like(b, float("nan"))
    Qe = torch.empty((len(snaps), 2), dtype=torch.float64, device="cuda")
    iters, res = ctx.solve_cg(b, q, Qe, tol=1e-13, maxit=1000)
    say(f"  iterations {iters}, residual {res:.2e}")
    assert 0 < iters < 1000 and res <= 1e-13
    _, bo, qo = _oracle(w, snaps[:5])
    assert rel(b.cpu().numpy()[:5], bo) < 1e-10
    qg = q.cpu().numpy()
    assert rel(qg[:5], qo) < 1e-10
    assert np.abs(qg.sum(axis=1)).max() <= 1e-12
    Qo = np.array([O.electrode_totals(x, w.electrode_id, 2) for x in qg])
    assert np.abs(Qe.cpu().numpy() - Qo).max() <= 1e-12 * max(1.0, np.abs(Qo).max())
    ctx.close()


def test_cg_paths_agree_with_direct_solve(cpm):
    """Operator CG, dense CG and the direct FP64 solve on the same b."""
    w = I.small_capacitor("b")
    say("cg vs direct small_capacitor_b")
    snaps = [0, 1, 2, 3]
    c1 = cpm.setup(w, matrix_free=True)
    c2 = cpm.setup(w)
    b = _b(c2, w, snaps)
    qd = torch.empty_like(b)
    c2.solve_charges(b, 0, qd)
    q1, q2 = torch.empty_like(b), torch.empty_like(b)
    c1.solve_cg(b, q1, tol=1e-13)
    c2.solve_cg(b, q2, tol=1e-13)
    qd = qd.cpu().numpy()
    assert rel(q1.cpu().numpy(), qd) < 1e-10
    assert rel(q2.cpu().numpy(), qd) < 1e-10
    c1.close()
    c2.close()


def test_cg_fp32_b_and_diag_extra(cpm):
    """FP32 b and a per-atom diagonal extra (the Thomas-Fermi-shaped term)."""
    w = I.small_capacitor("a")
    say("cg with FP32 b and diag_extra")
    diag = 0.05 + 0.01 * (np.arange(w.n) % 3)
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    ctx.build_operator(_dev(w.electrode_xyz), _dev(w.electrode_id, torch.int32), 2, _dev(diag))
    ctx.set_potential(w.v_electrode)
    b = _b(ctx, w, [0, 1], f32=True)
    q = torch.empty((2, w.n), dtype=torch.float64, device="cuda")
    ctx.solve_cg(b, q, tol=1e-13)
    p = O.params_for(w)
    A = O.elastance(w.electrode_xyz, p) + np.diag(diag)
    S = O.capacitance(A).S
    v = O.applied_potential(w.electrode_id, w.v_electrode)
    qo = np.array([O.charges(S, bb, v) for bb in b.double().cpu().numpy()])
    assert rel(q.cpu().numpy(), qo) < 1e-10
    assert np.abs(q.cpu().numpy().sum(axis=1)).max() <= 1e-12
    ctx.close()


def test_cg_finite_field_3d(cpm):
    """Tin-foil 3D cell with the finite-field potential -dv0 zeta (Eqs. 13-14)."""
    w = I.small_capacitor("a")
    Lz = 45.0
    say("cg finite field, 3D periodic")
    p = O.params_for(w, Lz=Lz, geometry="tinfoil")
    zeta = O.finite_field_zeta(w.electrode_xyz[:, 2], w.electrode_id, Lz)
    v = -1.5 * zeta
    gp = cpm.Params(w.Lx, w.Ly, Lz, 1.0, w.eta, w.alpha, w.rcut, w.kspace_eps, geometry=2)
    ctx = cpm.Context(gp)
    ctx.set_electrolyte(w.electrolyte_q)
    ctx.build_operator(_dev(w.electrode_xyz), _dev(w.electrode_id, torch.int32), 2)
    ctx.set_potential_atoms(v)
    b = _b(ctx, w, [2])
    q = torch.empty_like(b)
    ctx.solve_cg(b, q, tol=1e-13)
    _, bo, qo = _oracle(w, [2], p=p, v=v)
    assert rel(b.cpu().numpy(), bo) < 1e-10
    assert rel(q.cpu().numpy(), qo) < 1e-10
    assert abs(q.cpu().numpy().sum()) <= 1e-12
    ctx.close()


def test_cg_2880_against_golden(cpm):
    """2880-atom capacitor: operator columns against the stored oracle rows of
    A, and the CG charges against the stored oracle charges."""
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    g = dict(np.load(GOLDEN))
    w = I.graphite_capacitor()
    say(f"cg graphite_capacitor_2880 n={w.n}")
    ctx = cpm.setup(w, matrix_free=True)
    rows = g["rows"]
    X = np.zeros((len(rows), w.n))
    X[np.arange(len(rows)), rows] = 1.0
    Y = ctx.apply_elastance(_dev(X), torch.empty_like(_dev(X))).cpu().numpy()
    assert rel(Y, g["A_rows"]) < 1e-11
    assert rel(Y[np.arange(len(rows)), rows], g["A_diag"][rows]) < 1e-11
    snaps = [int(s) for s in g["snapshots"]]
    b = _b(ctx, w, snaps)
    q = torch.empty_like(b)
    Qe = torch.empty((len(snaps), 2), dtype=torch.float64, device="cuda")
    iters, res = ctx.solve_cg(b, q, Qe, tol=1e-13)
    say(f"  iterations {iters}, residual {res:.2e}, ELL width {ctx.info('ell_width'):.0f}")
    assert rel(q.cpu().numpy(), g["q"]) < 1e-10
    assert rel(Qe.cpu().numpy(), g["Q"]) < 1e-10
    assert np.abs(q.cpu().numpy().sum(axis=1)).max() <= 1e-12
    ctx.close()


def test_cg_limits_and_errors(cpm):
    w = I.small_capacitor("a")
    say("cg: iteration limit, empty batch, call order, unsupported electrodes")
    ctx = cpm.setup(w, matrix_free=True)
    b = _b(ctx, w, [0, 1])
    q = torch.empty_like(b)
    with pytest.raises(cpm.CpmError) as ei:
        ctx.solve_cg(b, q, tol=1e-13, maxit=3)
    assert ei.value.status == cpm.ENOCONV
    assert ctx.info("cg_iters") == 3 and ctx.info("cg_resid") > 1e-13
    assert np.isfinite(q.cpu().numpy()).all()
    assert np.abs(q.cpu().numpy().sum(axis=1)).max() <= 1e-12
    # tol = 0 with a zero right-hand side: nothing to do, q = 0
    z = torch.zeros_like(b)
    ctx.set_potential([0.0, 0.0])
    iters, res = ctx.solve_cg(z, q, tol=0.0, maxit=5)
    assert iters == 0 and res == 0.0 and not q.cpu().numpy().any()
    ctx.solve_cg(b[:0], q[:0])                    # empty batch: no-op
    with pytest.raises(cpm.CpmError) as ei:       # no S on an operator context
        ctx.solve_charges(b, 0, q)
    assert ei.value.status == cpm.ESTATE
    with pytest.raises(cpm.CpmError) as ei:
        ctx.invert(1)
    assert ei.value.status == cpm.ESTATE
    ctx.close()
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    ctx.build_operator(_dev(w.electrode_xyz), _dev(w.electrode_id, torch.int32), 2)
    with pytest.raises(cpm.CpmError) as ei:       # no potential yet
        ctx.solve_cg(b, q)
    assert ei.value.status == cpm.ESTATE
    with pytest.raises(cpm.CpmError) as ei:       # a context holds A or the operator
        ctx.build_elastance(_dev(w.electrode_xyz), _dev(w.electrode_id, torch.int32), 2)
    assert ei.value.status == cpm.ESTATE
    ctx.close()
    # electrodes off z planes (every atom its own z): no operator
    Rj = w.electrode_xyz + np.c_[np.zeros((w.n, 2)), 1e-3 * np.arange(w.n) / w.n]
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    with pytest.raises(cpm.CpmError) as ei:
        ctx.build_operator(_dev(Rj), _dev(w.electrode_id, torch.int32), 2)
    assert ei.value.status == cpm.EUNSUPPORTED
    ctx.close()


def test_cg_wire_tubes(cpm):
    """Co-axial tubes in the wire geometry (Eq. 11): the atoms share two z
    values per axial period, so the operator applies; many z images."""
    R, eid, R1, R2, per = I.coaxial_tubes(4, 8)
    Lxy = 2 * R2 + 40.0
    c = np.array([Lxy / 2, Lxy / 2, 0.0])
    R = R + c
    rad = 0.5 * (R1 + R2)
    ang = np.array([0.3, 1.9, 3.4, 5.0])
    r = np.column_stack([c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang),
                         np.array([0.2, 0.9, 1.5, 2.1])])
    qy = np.array([1.0, -1.0, 1.0, -1.0])
    say(f"cg wire tubes n={len(R)}")
    p = O.Params(Lxy, Lxy, per, eta=1.979, alpha=0.3, rcut=12.0, kspace_eps=1e-8, geometry="wire")
    A = O.elastance(R, p)
    S = O.capacitance(A).S
    v = O.applied_potential(eid, [-0.5, 0.5])
    bo = O.potential_vector(R, r, qy, p)
    qo = O.charges(S, bo, v)
    ctx = cpm.Context(cpm.Params(Lxy, Lxy, per, 1.0, 1.979, 0.3, 12.0, 1e-8, geometry=1))
    ctx.set_electrolyte(qy)
    ctx.build_operator(_dev(R), _dev(eid, torch.int32), 2)
    assert ctx.info("nlayers") == 2
    ctx.set_potential([-0.5, 0.5])
    X = np.eye(len(R))
    Y = ctx.apply_elastance(_dev(X), torch.empty_like(_dev(X))).cpu().numpy()
    assert rel(Y, A) < 1e-12
    b = torch.empty((1, len(R)), dtype=torch.float64, device="cuda")
    ctx.potential_vector(_dev(r[None]), b)
    q = torch.empty_like(b)
    ctx.solve_cg(b, q, tol=1e-13)
    assert rel(b.cpu().numpy()[0], bo) < 1e-10
    assert rel(q.cpu().numpy()[0], qo) < 1e-10
    assert abs(q.cpu().numpy().sum()) <= 1e-12
    ctx.close()


def test_cg_preconditioner_2880(cpm, monkeypatch):
    """The two-level preconditioner (smoother: inverse 64 x 64 diagonal tile
    blocks; coarse space: tile constants, or constants and in-plane offsets;
    additive form 1, balancing form 2) changes the iterates, not the
    solution: without it and in every form the charges of the 2880-atom
    capacitor (48 tiles: coarse arrays of 48 or 144 columns padded to 64 or
    192) match the stored oracle charges, and each variant takes fewer
    iterations than the one before."""
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_golden.py")
    g = dict(np.load(GOLDEN))
    w = I.graphite_capacitor()
    snaps = [int(s) for s in g["snapshots"]]
    iters = {}
    for pc, coarse in (("0", 1), ("1", 1), ("2", 1), ("2", 3)):
        monkeypatch.setenv("CPM_CG_PRECOND", pc)
        monkeypatch.setenv("CPM_CG_COARSE", str(coarse))
        say(f"cg graphite_capacitor_2880, preconditioner {pc}, coarse functions per tile {coarse}")
        ctx = cpm.setup(w, matrix_free=True)
        b = _b(ctx, w, snaps)
        q = torch.empty_like(b)
        Qe = torch.empty((len(snaps), 2), dtype=torch.float64, device="cuda")
        key = pc + str(coarse)
        iters[key], res = ctx.solve_cg(b, q, Qe, tol=1e-13)
        tiles, mode, ncoarse = ctx.info("pc_tiles"), ctx.info("pc_mode"), ctx.info("pc_coarse")
        say(f"  iterations {iters[key]}, residual {res:.2e}, tiles {tiles:.0f}, form {mode:.0f}, "
            f"coarse columns {ncoarse:.0f}")
        assert res <= 1e-13
        assert mode == int(pc) and tiles == (48 if pc != "0" else 0)
        assert ncoarse == tiles * coarse
        assert rel(q.cpu().numpy(), g["q"]) < 1e-10
        assert rel(Qe.cpu().numpy(), g["Q"]) < 1e-10
        assert np.abs(q.cpu().numpy().sum(axis=1)).max() <= 1e-12
        ctx.close()
    assert iters["23"] < iters["21"] < iters["11"] < iters["01"]


def test_operator_rebuild_with_other_plane_sizes(cpm):
    """A rebuild of the operator with the same n and number of planes but
    other atoms per plane (20 atoms of the lower layer moved, shifted off the
    upper layer's sites, into the upper plane: 124 + 164 atoms, so the atom
    map shrinks from 6 to 5 tiles) sizes the CG work, the preconditioner and
    the b-path work anew; b and the CG charges match the oracle for the new
    electrodes."""
    w = I.small_capacitor("a")
    say("operator rebuild with other plane sizes")
    ctx = cpm.setup(w, matrix_free=True)
    b = _b(ctx, w, [0, 1])
    q = torch.empty_like(b)
    ctx.solve_cg(b, q, tol=1e-13)
    tiles0 = ctx.info("pc_tiles")
    R = w.electrode_xyz.copy()
    low = np.where(R[:, 2] == R[:, 2].min())[0][:20]
    R[low] += np.array([0.31, 0.43, 30.0])
    ctx.build_operator(_dev(R), _dev(w.electrode_id, torch.int32), 2)
    ctx.set_potential(w.v_electrode)
    xyz = _dev(np.stack([I.snapshot(w, s) for s in (0, 1)]))
    b2 = torch.empty_like(b)
    ctx.potential_vector(xyz, b2)
    iters, res = ctx.solve_cg(b2, q, tol=1e-13)
    say(f"  tiles {tiles0:.0f} -> {ctx.info('pc_tiles'):.0f}, iterations {iters}")
    assert tiles0 == 6 and ctx.info("pc_tiles") == 5
    p = O.params_for(w)
    A = O.elastance(R, p)
    S = O.capacitance(A).S
    v = O.applied_potential(w.electrode_id, w.v_electrode)
    bo = np.array([O.potential_vector(R, I.snapshot(w, s), w.electrolyte_q, p) for s in (0, 1)])
    assert rel(b2.cpu().numpy(), bo) < 1e-10
    qo = np.array([O.charges(S, x, v) for x in bo])
    assert rel(q.cpu().numpy(), qo) < 1e-10
    assert np.abs(q.cpu().numpy().sum(axis=1)).max() <= 1e-12
    ctx.close()


def test_cg_iteration_graphs_match_eager(cpm, monkeypatch):
    """The 8-iteration blocks of the CG replayed as HIP graphs (the context's
    own stream, or the internal stream of a NULL-stream context) give the
    same charges, bit for bit, as eager launches; two groups (35 vectors) and
    two calls, so the graphs are replayed many times with eager kernels and
    host checks in between, and a second tolerance captures anew."""
    w = I.graphite_capacitor()
    snaps = list(range(35))
    out = {}
    for name, env, use_stream in (("eager", "0", False), ("null", "1", False), ("own", "1", True)):
        monkeypatch.setenv("CPM_CG_GRAPH", env)
        say(f"cg iteration graphs: {name}")
        stream = torch.cuda.Stream() if use_stream else None
        ctx = cpm.setup(w, matrix_free=True, stream=stream)
        b = _b(ctx, w, snaps)
        if stream is not None:
            stream.synchronize()
        res = []
        for tol in (1e-13, 1e-13, 1e-10):
            q = torch.empty_like(b)
            iters, r = ctx.solve_cg(b, q, tol=tol)
            res.append((iters, q.cpu().numpy()))
        out[name] = res
        ctx.close()
    for name in ("null", "own"):
        for (i0, q0), (i1, q1) in zip(out["eager"], out[name]):
            assert i0 == i1
            assert np.array_equal(q0, q1), name
    g = dict(np.load(GOLDEN)) if os.path.exists(GOLDEN) else None
    if g is not None:
        idx = [snaps.index(int(s)) for s in g["snapshots"] if int(s) in snaps]
        if idx:
            assert rel(out["null"][0][1][idx], g["q"][:len(idx)]) < 1e-10


def test_cg_large_coarse_space_matches_direct(cpm):
    """8400-atom capacitor (132 tiles): the balancing form takes the in-plane
    offsets into its coarse space by itself (396 coarse functions, so the
    coarse products run split over the coarse columns); its charges match
    the direct FP64 solve q = S (b + v) on the same b, which the 2880-atom
    case ties to the oracle, and the oracle's own sampled rows of b and A."""
    w = I.scaled_graphite_capacitor(8500)
    say(f"cg with the large coarse space, n={w.n}")
    direct = cpm.setup(w)
    ctx = cpm.setup(w, matrix_free=True)
    b = _b(direct, w, [0, 1, 2])
    qd = torch.empty_like(b)
    direct.solve_charges(b, 0, qd)
    q = torch.empty_like(b)
    iters, res = ctx.solve_cg(b, q, tol=1e-13)
    tiles, ncoarse = ctx.info("pc_tiles"), ctx.info("pc_coarse")
    say(f"  iterations {iters}, tiles {tiles:.0f}, coarse functions {ncoarse:.0f}")
    assert tiles == 132 and ncoarse == 3 * 132 and ctx.info("pc_mode") == 2
    assert rel(q.cpu().numpy(), qd.cpu().numpy()) < 1e-10
    assert np.abs(q.cpu().numpy().sum(axis=1)).max() <= 1e-12
    # against the oracle's stored rows of b and A for snapshots 0-2: b rows at
    # 1e-10, and A q - b - v uniform on every stored row
    gl = np.load(os.path.join(os.path.dirname(GOLDEN), "scaled_graphite_capacitor_8400_rows_alpha0.30.npz"))
    rows, qc, bc = gl["rows"], q.cpu().numpy(), b.cpu().numpy()
    assert rel(bc[:, rows], gl["b_rows"]) < 1e-10
    for s in range(3):
        r = gl["A_rows"] @ qc[s] - gl["b_rows"][s] - gl["v_rows"]
        assert np.abs(r - r.mean()).max() <= 1e-10 * np.abs(gl["b_rows"][s] + gl["v_rows"]).max()
    direct.close()
    ctx.close()
