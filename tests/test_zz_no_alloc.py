"""cpm_solve_charges_noalloc against cpm_solve_charges through the C-ABI.

The allocation-free entry point keeps its work buffers in the library's
fixed scratch array.  On the same b it must give the charges the ordinary
entry point gives, to the path's tolerance (1e-10 relative for FP64 and
1e-5 for the refined FP32 / split-BF16 modes; the kernels and launch shapes
are the same, so the results are expected to be equal), on two calls in a
row, the second with a smaller batch, whose shared scratch still holds the
first call's contents.
"""
import sys

import numpy as np
import pytest

from paper_2203_15461_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cpm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_15461_amd import cpm as C
    C.lib()
    return C


def _b(ctx, w, count, f32):
    xyz = torch.as_tensor(np.stack([I.snapshot(w, s) for s in range(count)]), dtype=torch.float64,
                          device="cuda").contiguous()
    b = torch.empty((count, w.n), dtype=torch.float32 if f32 else torch.float64, device="cuda")
    ctx.potential_vector(xyz, b)
    return b


@pytest.mark.parametrize("mode,batches,tol", [
    (0x000, (3, 1), 1e-10),        # FP64 streaming matvec
    (0x000, (40, 8), 1e-10),       # FP64 matrix-core product
    (0x101, (3, 2), 1e-5),         # FP32 S + FP64 refinement (matvecs)
    (0x102, (100, 8), 1e-5),       # split-BF16 product + FP64 refinement
])
def test_noalloc_matches_solve_charges(cpm, mode, batches, tol):
    w = I.graphite_capacitor()
    f32 = (mode & 0xff) == 1
    say(f"noalloc mode {mode:#x} batches {batches} n={w.n}")
    ctx = cpm.setup(w, store=cpm.STORE_F64 | cpm.STORE_F32 | cpm.STORE_BF16X2)
    b_all = _b(ctx, w, max(batches), f32)
    for batch in batches:                       # the second call is smaller
        b = b_all[:batch].contiguous()
        q_ref = torch.empty((batch, w.n), dtype=torch.float64, device="cuda")
        Q_ref = torch.empty((batch, 2), dtype=torch.float64, device="cuda")
        ctx.solve_charges(b, mode, q_ref, Q_ref)
        q = torch.full((batch, w.n), float("nan"), dtype=torch.float64, device="cuda")
        Q = torch.full((batch, 2), float("nan"), dtype=torch.float64, device="cuda")
        ctx.solve_charges_noalloc(b, mode, q, Q)
        ctx.synchronize()
        qr, qn = q_ref.cpu().numpy(), q.cpu().numpy()
        err = float(np.abs(qn - qr).max() / np.abs(qr).max())
        say(f"  batch {batch}: max rel diff {err:.3e}")
        assert err <= tol
        assert np.abs(Q.cpu().numpy() - Q_ref.cpu().numpy()).max() <= tol * np.abs(Q_ref.cpu().numpy()).max()
        assert np.all(np.abs(qn.sum(1)) <= 1e-12)
    ctx.close()


def test_noalloc_rejects_too_large_batch(cpm):
    w = I.graphite_capacitor()
    say("noalloc size limit")
    ctx = cpm.setup(w, store=cpm.STORE_F64 | cpm.STORE_BF16X2)
    b = torch.zeros((200, w.n), dtype=torch.float64, device="cuda")
    q = torch.empty_like(b)
    with pytest.raises(cpm.CpmError) as ei:       # 256 padded rows exceed 16 MiB at n = 2880
        ctx.solve_charges_noalloc(b, 0x102, q)
    assert ei.value.status == cpm.EINVAL
    assert "scratch" in str(ei.value)
    ctx.close()
