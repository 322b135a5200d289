"""Thin ctypes binding of libcpm (include/cpm.h).

Argument marshalling only: device memory comes from torch tensors, the HIP
stream from torch's current stream, and every step of the charge solve runs
in the library's HIP kernels.  There is no CPU fallback: if libcpm.so is not
built, `lib()` raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpm.so")

# status codes
OK, EINVAL, ESTATE, ENOMEM, EHIP, ENOTPD, EUNSUPPORTED, ENOCONV = range(8)
STATUS_NAMES = {0: "CPM_OK", 1: "CPM_EINVAL", 2: "CPM_ESTATE", 3: "CPM_ENOMEM", 4: "CPM_EHIP",
                5: "CPM_ENOTPD", 6: "CPM_EUNSUPPORTED", 7: "CPM_ENOCONV"}
# store flags, solve modes, info keys
STORE_F64, STORE_F32, STORE_BF16X2 = 1, 2, 4
INVERT_ASYNC = 0x100
INVERT_FACTOR = 0x200
SOLVE_F64, SOLVE_F32, SOLVE_BF16X2, SOLVE_REFINE, SOLVE_CCM = 0, 1, 2, 0x100, 0x200
INFO = dict(n=0, nk=1, ne=2, s_sum=3, pivot=4, lz=5, kcut=6, m=7, workspace=8, npad=9, nruns=10,
            nlayers=11, sf_matrix=12, tune_bm=13, tune_ks=14, tune_grid=15, tune_us=16, group=17,
            cg_iters=18, cg_resid=19, ell_width=20, ncols=21,
            bsr_blocks=22, pc_tiles=23, pc_mode=24, pc_coarse=25, sf_fp32=26, rs_plane=27)

EXPORTS = ("cpm_create", "cpm_set_electrolyte", "cpm_build_elastance", "cpm_invert",
           "cpm_set_potential", "cpm_potential_vector", "cpm_solve_charges", "cpm_copy_matrix",
           "cpm_copy_vector", "cpm_capture_step", "cpm_replay_step", "cpm_autotune",
           "cpm_solve_grouped", "cpm_capture_grouped", "cpm_replay_grouped", "cpm_set_charge", "cpm_set_potential_atoms", "cpm_build_operator",
           "cpm_apply_elastance", "cpm_solve_cg", "cpm_get_info",
           "cpm_enable_timing", "cpm_get_timing", "cpm_set_field", "cpm_save", "cpm_load",
           "cpm_inspect_file", "cpm_solve_charges_noalloc",
           "cpm_synchronize", "cpm_last_error", "cpm_destroy")


class CpmParams(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("h", ctypes.c_double),
                ("slab_factor", ctypes.c_double), ("eta", ctypes.c_double),
                ("alpha", ctypes.c_double), ("rcut", ctypes.c_double),
                ("kspace_eps", ctypes.c_double), ("kcut", ctypes.c_double),
                ("coulomb_k", ctypes.c_double), ("geometry", ctypes.c_int)]


class CpmFileInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_e", ctypes.c_int), ("matrices", ctypes.c_int),
                ("store", ctypes.c_uint), ("geometry_hash", ctypes.c_ulonglong),
                ("s_sum", ctypes.c_double), ("params", CpmParams)]


NOALLOC_SCRATCH_BYTES = 16 << 20


class CpmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def lib(path: str | None = None) -> ctypes.CDLL:
    """Open libcpm.so (built by paper_2203_15461_amd.build); raise if absent."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run `python -m paper_2203_15461_amd.build`")
    L = ctypes.CDLL(p)
    vp, i, d, u = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    sig = {
        "cpm_create": ([ctypes.POINTER(CpmParams), vp, ctypes.POINTER(vp)], i),
        "cpm_set_electrolyte": ([vp, i, vp], i),
        "cpm_build_elastance": ([vp, i, vp, vp, i, vp], i),
        "cpm_build_operator": ([vp, i, vp, vp, i, vp], i),
        "cpm_solve_cg": ([vp, i, vp, i, d, i, vp, vp], i),
        "cpm_apply_elastance": ([vp, i, vp, vp], i),
        "cpm_invert": ([vp, u], i),
        "cpm_set_potential": ([vp, vp], i),
        "cpm_potential_vector": ([vp, i, vp, vp, i], i),
        "cpm_solve_charges": ([vp, i, vp, i, u, vp, vp], i),
        "cpm_copy_matrix": ([vp, i, vp], i),
        "cpm_capture_step": ([vp, i, vp, vp, i, u, vp, vp], i),
        "cpm_replay_step": ([vp], i),
        "cpm_autotune": ([vp, i, i], i),
        "cpm_set_charge": ([vp, ctypes.POINTER(d)], i),
        "cpm_set_potential_atoms": ([vp, ctypes.POINTER(d)], i),
        "cpm_solve_grouped": ([ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(vp), i, u,
                               ctypes.POINTER(vp), ctypes.POINTER(vp)], i),
        "cpm_capture_grouped": ([ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(vp),
                                 ctypes.POINTER(vp), i, u, ctypes.POINTER(vp), ctypes.POINTER(vp)], i),
        "cpm_replay_grouped": ([ctypes.POINTER(vp), i], i),
        "cpm_copy_vector": ([vp, i, vp], i),
        "cpm_get_info": ([vp, i, ctypes.POINTER(d)], i),
        "cpm_enable_timing": ([vp, ctypes.c_char_p], i),
        "cpm_get_timing": ([vp, ctypes.c_char_p, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_longlong)], i),
        "cpm_synchronize": ([vp], i),
        "cpm_set_field": ([vp, d, i], i),
        "cpm_save": ([vp, ctypes.c_char_p], i),
        "cpm_load": ([vp, ctypes.c_char_p], i),
        "cpm_inspect_file": ([ctypes.c_char_p, ctypes.POINTER(CpmFileInfo)], i),
        "cpm_solve_charges_noalloc": ([vp, i, vp, i, u, vp, vp], i),
        "cpm_last_error": ([vp], ctypes.c_char_p),
        "cpm_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _LIB = L
    return L


@dataclass
class Params:
    """Method knobs (cpm_params).  Lz = slab_factor * h."""
    Lx: float
    Ly: float
    h: float
    slab_factor: float = 3.0
    eta: float = 1.979
    alpha: float = 0.3
    rcut: float = 12.0
    kspace_eps: float = 1e-8
    kcut: float = 0.0
    coulomb_k: float = 0.0
    geometry: int = 0

    def to_c(self) -> CpmParams:
        return CpmParams(self.Lx, self.Ly, self.h, self.slab_factor, self.eta, self.alpha,
                         self.rcut, self.kspace_eps, self.kcut, self.coulomb_k, self.geometry)

    @staticmethod
    def of(w) -> "Params":
        return Params(w.Lx, w.Ly, w.h, w.slab_factor, w.eta, w.alpha, w.rcut, w.kspace_eps)


def _ptr(t) -> ctypes.c_void_p | None:
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """One CPM charge-solve context on one HIP stream (see include/cpm.h)."""

    def __init__(self, params: Params, stream=None):
        self._lib = lib()
        self._h = ctypes.c_void_p()
        self._stream = stream
        p = params.to_c()
        st = self._lib.cpm_create(ctypes.byref(p), _stream_handle(stream), ctypes.byref(self._h))
        if st != OK:
            raise CpmError(st, "cpm_create rejected the parameters")
        self.params = params

    # -- plumbing -----------------------------------------------------------
    def _check(self, st: int, what: str):
        if st != OK:
            msg = self._lib.cpm_last_error(self._h).decode(errors="replace")
            raise CpmError(st, f"{what}: {msg}")

    def close(self):
        if self._h:
            self._lib.cpm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, key: str) -> float:
        out = ctypes.c_double()
        self._check(self._lib.cpm_get_info(self._h, INFO[key], ctypes.byref(out)), "cpm_get_info")
        return out.value

    def enable_timing(self, on=True):
        """Per-kernel-family HIP event timing on the context stream (clears totals).

        on: True (every family), False/None (off), or an iterable / comma-separated
        string of family names to time only those."""
        if on is True:
            spec = b"*"
        elif not on:
            spec = None
        elif isinstance(on, str):
            spec = on.encode()
        else:
            spec = ",".join(on).encode()
        self._check(self._lib.cpm_enable_timing(self._h, spec), "cpm_enable_timing")

    def timing(self, name: str):
        """(total_ms, launches) of one kernel family since timing was enabled."""
        ms, cnt = ctypes.c_double(), ctypes.c_longlong()
        self._check(self._lib.cpm_get_timing(self._h, name.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
                    "cpm_get_timing")
        return ms.value, cnt.value

    def synchronize(self):
        self._check(self._lib.cpm_synchronize(self._h), "cpm_synchronize")

    # -- the C-ABI entry points --------------------------------------------
    def set_electrolyte(self, q):
        """Electrolyte charges (host array-like of float64), fixed for the run."""
        import numpy as np
        qa = np.ascontiguousarray(q, dtype=np.float64)
        self._check(self._lib.cpm_set_electrolyte(self._h, len(qa), qa.ctypes.data_as(ctypes.c_void_p)),
                    "cpm_set_electrolyte")

    def build_elastance(self, xyz, eid, n_e: int, diag_extra=None):
        """xyz: (n, 3) float64 CUDA tensor; eid: (n,) int32 CUDA tensor."""
        self._build("cpm_build_elastance", xyz, eid, n_e, diag_extra)

    def build_operator(self, xyz, eid, n_e: int, diag_extra=None):
        """The matrix-free elastance operator (same arguments as build_elastance)."""
        self._build("cpm_build_operator", xyz, eid, n_e, diag_extra)

    def _build(self, fn, xyz, eid, n_e, diag_extra):
        _expect(xyz, "float64", 2)
        _expect(eid, "int32", 1)
        if xyz.shape[1] != 3 or eid.shape[0] != xyz.shape[0]:
            raise ValueError("xyz must be (n, 3) and eid (n,)")
        if diag_extra is not None:
            _expect(diag_extra, "float64", 1)
            if diag_extra.shape[0] != xyz.shape[0]:
                raise ValueError("diag_extra must be (n,)")
        self._check(getattr(self._lib, fn)(self._h, xyz.shape[0], _ptr(xyz), _ptr(eid), n_e,
                                           _ptr(diag_extra)), fn)

    def invert(self, store: int = STORE_F64):
        self._check(self._lib.cpm_invert(self._h, store), "cpm_invert")

    def set_potential(self, v_electrode):
        """One potential (V) per electrode."""
        import numpy as np
        va = np.ascontiguousarray(v_electrode, dtype=np.float64).ravel()
        if len(va) != int(self.info("ne")):
            raise ValueError(f"need {int(self.info('ne'))} electrode potentials, got {len(va)}")
        self._check(self._lib.cpm_set_potential(self._h, va.ctypes.data_as(ctypes.c_void_p)),
                    "cpm_set_potential")

    def set_potential_atoms(self, v_atoms):
        """One potential (V) per electrode atom (e.g. the finite-field -dv0 zeta)."""
        import numpy as np
        va = np.ascontiguousarray(v_atoms, dtype=np.float64).ravel()
        if len(va) != int(self.info("n")):
            raise ValueError(f"need {int(self.info('n'))} atom potentials, got {len(va)}")
        self._check(self._lib.cpm_set_potential_atoms(
            self._h, va.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "cpm_set_potential_atoms")

    def set_field(self, dv0: float, bottom: int = 0):
        """Finite-field potential -dv0 zeta, zeta formed by the library from the
        electrode z coordinates (3D-periodic cell; `bottom` gets the +1 offset)."""
        self._check(self._lib.cpm_set_field(self._h, float(dv0), int(bottom)), "cpm_set_field")

    def save(self, path: str):
        """Write A (and A^-1 after invert) with the geometry fingerprint."""
        self._check(self._lib.cpm_save(self._h, os.fsencode(path)), "cpm_save")

    def load(self, path: str):
        """Read a state file written for the same electrodes and knobs."""
        self._check(self._lib.cpm_load(self._h, os.fsencode(path)), "cpm_load")

    def set_charge(self, Q_electrode):
        """Constrained charge method: total charge (e) per electrode, summing to zero."""
        import numpy as np
        Qa = np.ascontiguousarray(Q_electrode, dtype=np.float64).ravel()
        if len(Qa) != int(self.info("ne")):
            raise ValueError(f"need {int(self.info('ne'))} electrode charges, got {len(Qa)}")
        self._check(self._lib.cpm_set_charge(self._h, Qa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "cpm_set_charge")

    def potential_vector(self, xyz, out):
        """xyz: (batch, m, 3) float64 CUDA tensor; out: (batch, n) float64 or float32."""
        _expect(xyz, "float64", 3)
        f32 = _is_f32(out)
        n, m = int(self.info("n")), int(self.info("m"))
        if tuple(xyz.shape[1:]) != (m, 3) or tuple(out.shape) != (xyz.shape[0], n):
            raise ValueError(f"shapes {tuple(xyz.shape)}, {tuple(out.shape)} do not match m={m}, n={n}")
        self._check(self._lib.cpm_potential_vector(self._h, xyz.shape[0], _ptr(xyz), _ptr(out), f32),
                    "cpm_potential_vector")
        return out

    def solve_charges(self, b, mode: int, q_out, Qe_out=None):
        """b: (batch, n) float64/float32; q_out: (batch, n) float64; Qe_out: (batch, n_e) or None."""
        _expect(q_out, "float64", 2)
        f32 = _is_f32(b)
        n, ne = int(self.info("n")), int(self.info("ne"))
        if n == 0:   # no elastance yet: the library reports the call-order error
            self._check(self._lib.cpm_solve_charges(self._h, b.shape[0], _ptr(b), f32, mode,
                                                    _ptr(q_out), _ptr(Qe_out)), "cpm_solve_charges")
        if b.dim() != 2 or tuple(b.shape) != tuple(q_out.shape) or b.shape[1] != n:
            raise ValueError(f"b {tuple(b.shape)} and q {tuple(q_out.shape)} must both be (batch, {n})")
        if Qe_out is not None:
            _expect(Qe_out, "float64", 2)
            if tuple(Qe_out.shape) != (b.shape[0], ne):
                raise ValueError(f"Qe must be (batch, {ne})")
        self._check(self._lib.cpm_solve_charges(self._h, b.shape[0], _ptr(b), f32, mode, _ptr(q_out),
                                                _ptr(Qe_out)), "cpm_solve_charges")
        return q_out

    def solve_charges_noalloc(self, b, mode: int, q_out, Qe_out=None):
        """cpm_solve_charges with the work buffers in the library's fixed
        scratch array (allocates nothing)."""
        _expect(q_out, "float64", 2)
        f32 = _is_f32(b)
        n, ne = int(self.info("n")), int(self.info("ne"))
        if b.dim() != 2 or tuple(b.shape) != tuple(q_out.shape) or b.shape[1] != n:
            raise ValueError(f"b {tuple(b.shape)} and q {tuple(q_out.shape)} must both be (batch, {n})")
        if Qe_out is not None:
            _expect(Qe_out, "float64", 2)
            if tuple(Qe_out.shape) != (b.shape[0], ne):
                raise ValueError(f"Qe must be (batch, {ne})")
        self._check(self._lib.cpm_solve_charges_noalloc(self._h, b.shape[0], _ptr(b), f32, mode,
                                                        _ptr(q_out), _ptr(Qe_out)),
                    "cpm_solve_charges_noalloc")
        return q_out

    def apply_elastance(self, x, y_out):
        """y = A x for x (batch, n) float64 (operator or dense A)."""
        _expect(x, "float64", 2)
        _expect(y_out, "float64", 2)
        if tuple(x.shape) != tuple(y_out.shape) or x.shape[1] != int(self.info("n")):
            raise ValueError("x and y must both be (batch, n)")
        self._check(self._lib.cpm_apply_elastance(self._h, x.shape[0], _ptr(x), _ptr(y_out)),
                    "cpm_apply_elastance")
        return y_out

    def solve_cg(self, b, q_out, Qe_out=None, tol: float = 1e-13, maxit: int = 1000):
        """Conjugate-gradient charges: b (batch, n) float64/float32, q_out (batch, n)
        float64, Qe_out (batch, n_e) or None.  Returns (iterations, residual)."""
        _expect(q_out, "float64", 2)
        f32 = _is_f32(b)
        n, ne = int(self.info("n")), int(self.info("ne"))
        if n and (b.dim() != 2 or tuple(b.shape) != tuple(q_out.shape) or b.shape[1] != n):
            raise ValueError(f"b {tuple(b.shape)} and q {tuple(q_out.shape)} must both be (batch, {n})")
        if Qe_out is not None:
            _expect(Qe_out, "float64", 2)
            if tuple(Qe_out.shape) != (b.shape[0], ne):
                raise ValueError(f"Qe must be (batch, {ne})")
        self._check(self._lib.cpm_solve_cg(self._h, b.shape[0], _ptr(b), f32, float(tol), int(maxit),
                                           _ptr(q_out), _ptr(Qe_out)), "cpm_solve_cg")
        return int(self.info("cg_iters")), self.info("cg_resid")

    def autotune(self, batch: int, reps: int = 5) -> dict:
        """Time the split-BF16 batched product's tile shapes for `batch` vectors;
        later solves with the same padded row count use the fastest."""
        self._check(self._lib.cpm_autotune(self._h, int(batch), int(reps)), "cpm_autotune")
        return {k: self.info("tune_" + k) for k in ("bm", "ks", "grid", "us")}

    def capture_step(self, xyz, b, mode: int, q_out, Qe_out=None):
        """Capture b for xyz (batch, m, 3) and the solve into a HIP graph."""
        _expect(xyz, "float64", 3)
        _expect(q_out, "float64", 2)
        f32 = _is_f32(b)
        n, m = int(self.info("n")), int(self.info("m"))
        if tuple(xyz.shape[1:]) != (m, 3) or tuple(b.shape) != (xyz.shape[0], n) \
                or tuple(q_out.shape) != (xyz.shape[0], n):
            raise ValueError("capture_step: shapes do not match (batch, m, 3), (batch, n)")
        if Qe_out is not None:
            _expect(Qe_out, "float64", 2)
            if tuple(Qe_out.shape) != (xyz.shape[0], int(self.info("ne"))):
                raise ValueError("capture_step: Qe must be (batch, n_e)")
        self._check(self._lib.cpm_capture_step(self._h, xyz.shape[0], _ptr(xyz), _ptr(b), f32, mode,
                                               _ptr(q_out), _ptr(Qe_out)), "cpm_capture_step")

    def replay_step(self):
        self._check(self._lib.cpm_replay_step(self._h), "cpm_replay_step")

    def copy_matrix(self, which: int, out):
        """which 0: A, 1: A^-1, 2: S into an (n, n) float64 tensor."""
        _expect(out, "float64", 2)
        n = int(self.info("n"))
        if tuple(out.shape) != (n, n):
            raise ValueError(f"need an ({n}, {n}) tensor")
        self._check(self._lib.cpm_copy_matrix(self._h, which, _ptr(out)), "cpm_copy_matrix")
        return out

    def copy_vector(self, which: int, out):
        """which 0: u = A^-1 e, 1: d = S v into an (n,) float64 tensor."""
        _expect(out, "float64", 1)
        if out.shape[0] != int(self.info("n")):
            raise ValueError("need an (n,) tensor")
        self._check(self._lib.cpm_copy_vector(self._h, which, _ptr(out)), "cpm_copy_vector")
        return out


def inspect_file(path: str) -> dict:
    """Header of a state file written by cpm_save (host only)."""
    out = CpmFileInfo()
    st = lib().cpm_inspect_file(os.fsencode(path), ctypes.byref(out))
    if st != OK:
        raise CpmError(st, f"cpm_inspect_file: {path} is not a valid state file")
    p = out.params
    return dict(n=out.n, n_e=out.n_e, matrices=out.matrices, store=out.store,
                geometry_hash=out.geometry_hash, s_sum=out.s_sum,
                params=dict(Lx=p.Lx, Ly=p.Ly, h=p.h, slab_factor=p.slab_factor, eta=p.eta,
                            alpha=p.alpha, rcut=p.rcut, kspace_eps=p.kspace_eps, kcut=p.kcut,
                            coulomb_k=p.coulomb_k, geometry=p.geometry))


def solve_grouped(ctxs, bs, mode: int, qs, Qes=None):
    """cpm_solve_grouped: one split-BF16 solve over several contexts (sharing one
    stream); bs[i] (batch_i, n_i), qs[i] (batch_i, n_i), Qes[i] (batch_i, n_e_i) or None."""
    k = len(ctxs)
    if not (len(bs) == len(qs) == k) or (Qes is not None and len(Qes) != k):
        raise ValueError("one b, q (and Qe) per context")
    f32 = {_is_f32(b) for b in bs}
    if len(f32) != 1:
        raise ValueError("all b must have the same dtype")
    for c, b, q, i in zip(ctxs, bs, qs, range(k)):
        _expect(q, "float64", 2)
        n, ne = int(c.info("n")), int(c.info("ne"))
        if b.dim() != 2 or tuple(b.shape) != tuple(q.shape) or b.shape[1] != n:
            raise ValueError(f"context {i}: b and q must both be (batch, {n})")
        if Qes is not None and Qes[i] is not None:
            _expect(Qes[i], "float64", 2)
            if tuple(Qes[i].shape) != (b.shape[0], ne):
                raise ValueError(f"context {i}: Qe must be (batch, {ne})")
    vp = ctypes.c_void_p
    H = (vp * k)(*[c._h.value for c in ctxs])
    Bt = (ctypes.c_int * k)(*[b.shape[0] for b in bs])
    Bp = (vp * k)(*[_ptr(b) for b in bs])
    Qp = (vp * k)(*[_ptr(q) for q in qs])
    Ep = (vp * k)(*[_ptr(e) for e in Qes]) if Qes is not None else None
    st = lib().cpm_solve_grouped(H, k, Bt, Bp, f32.pop(), mode, Qp, Ep)
    if st != OK:
        raise CpmError(st, "cpm_solve_grouped: " + lib().cpm_last_error(ctxs[0]._h).decode(errors="replace"))
    return qs


def _group_args(ctxs, bs, qs, Qes):
    """Shared checks and ctypes arrays of the grouped calls."""
    k = len(ctxs)
    if not (len(bs) == len(qs) == k) or (Qes is not None and len(Qes) != k):
        raise ValueError("one b, q (and Qe) per context")
    f32 = {_is_f32(b) for b in bs}
    if len(f32) != 1:
        raise ValueError("all b must have the same dtype")
    for c, b, q, i in zip(ctxs, bs, qs, range(k)):
        _expect(q, "float64", 2)
        n, ne = int(c.info("n")), int(c.info("ne"))
        if b.dim() != 2 or tuple(b.shape) != tuple(q.shape) or b.shape[1] != n:
            raise ValueError(f"context {i}: b and q must both be (batch, {n})")
        if Qes is not None and Qes[i] is not None:
            _expect(Qes[i], "float64", 2)
            if tuple(Qes[i].shape) != (b.shape[0], ne):
                raise ValueError(f"context {i}: Qe must be (batch, {ne})")
    vp = ctypes.c_void_p
    H = (vp * k)(*[c._h.value for c in ctxs])
    Bt = (ctypes.c_int * k)(*[b.shape[0] for b in bs])
    Bp = (vp * k)(*[_ptr(b) for b in bs])
    Qp = (vp * k)(*[_ptr(q) for q in qs])
    Ep = (vp * k)(*[_ptr(e) for e in Qes]) if Qes is not None else None
    return k, H, Bt, Bp, f32.pop(), Qp, Ep


def capture_grouped(ctxs, xyzs, bs, mode: int, qs, Qes=None):
    """cpm_capture_grouped: b of every context and their grouped solve as one
    HIP graph (contexts sharing one non-default stream); xyzs[i]
    (batch_i, m_i, 3) float64, bs/qs/Qes as for solve_grouped."""
    if len(xyzs) != len(ctxs):
        raise ValueError("one coordinate tensor per context")
    for c, x, b, i in zip(ctxs, xyzs, bs, range(len(ctxs))):
        _expect(x, "float64", 3)
        if tuple(x.shape) != (b.shape[0], int(c.info("m")), 3):
            raise ValueError(f"context {i}: xyz must be (batch, m, 3)")
    k, H, Bt, Bp, f32, Qp, Ep = _group_args(ctxs, bs, qs, Qes)
    Xp = (ctypes.c_void_p * k)(*[_ptr(x) for x in xyzs])
    st = lib().cpm_capture_grouped(H, k, Bt, Xp, Bp, f32, mode, Qp, Ep)
    if st != OK:
        raise CpmError(st, "cpm_capture_grouped: " + lib().cpm_last_error(ctxs[0]._h).decode(errors="replace"))


def replay_grouped(ctxs):
    """cpm_replay_grouped: launch the captured grouped step (asynchronous)."""
    H = (ctypes.c_void_p * len(ctxs))(*[c._h.value for c in ctxs])
    st = lib().cpm_replay_grouped(H, len(ctxs))
    if st != OK:
        raise CpmError(st, "cpm_replay_grouped: " + lib().cpm_last_error(ctxs[0]._h).decode(errors="replace"))


def _expect(t, dtype: str, ndim: int):
    if not t.is_cuda:
        raise ValueError("expected a device (HIP) tensor")
    if str(t.dtype) != "torch." + dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if t.dim() != ndim or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {ndim}-d tensor")


def _is_f32(t) -> int:
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if str(t.dtype) == "torch.float32":
        return 1
    if str(t.dtype) == "torch.float64":
        return 0
    raise ValueError(f"expected float32 or float64, got {t.dtype}")


def setup(w, store: int = STORE_F64, stream=None, params: Params | None = None,
          v_electrode=None, matrix_free: bool = False) -> Context:
    """Create a context for a generated workload: electrolyte charges, A, S, v
    (matrix_free: the elastance operator for solve_cg instead of A and S)."""
    import torch
    ctx = Context(params or Params.of(w), stream)
    ctx.set_electrolyte(w.electrolyte_q)
    xyz = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device="cuda").contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device="cuda").contiguous()
    if stream is not None:      # the copies above ran on torch's current stream
        torch.cuda.current_stream().synchronize()
    if matrix_free:
        ctx.build_operator(xyz, eid, int(w.electrode_id.max()) + 1)
    else:
        ctx.build_elastance(xyz, eid, int(w.electrode_id.max()) + 1)
        ctx.invert(store)
    ctx.set_potential(w.v_electrode if v_electrode is None else v_electrode)
    return ctx
