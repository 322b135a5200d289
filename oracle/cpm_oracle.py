"""Plain FP64 CPU oracle for the constant-potential-method (CPM) charge solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path (the
HIP library and its binding) never calls it and shares no code with it.

What is computed (ELECTRODE paper, Sec. II.A, II.B, II.E):

* Electrode atoms i carry Gaussian charges of reciprocal width eta
  (Sec. III.B, the definition of rho_i).  Two such Gaussians interact through
  erf(eta_ee r)/r with eta_ee = eta/sqrt(2); a Gaussian and an electrolyte
  point charge interact through erf(eta r)/r.
* The electrode Coulomb energy is U = 1/2 q^T A q - b^T q - v^T q (Eq. 2).
  A is the elastance matrix (electrode-electrode, periodic images included),
  b is minus the electrolyte potential at the electrode atoms.
* With total charge held at zero the minimiser is q = S (b + v), with
  S = A^-1 - A^-1 e e^T A^-1 / (e^T A^-1 e) (Eqs. 3, 4); v = G v~ (Eqs. 5, 6).
* Slab geometry adds the EW3DC dipole energy (2 pi/V) M_z^2 (Eq. 10), split
  into an electrode part (into A) and an electrolyte cross term (into b)
  (Eq. 12).  The 1D-periodic variant (pi/V)(M_x^2 + M_y^2) (Eq. 11) is here
  too, for the co-axial capacitor check of Sec. III.B.

The Ewald split of the periodic sums is the textbook one (the paper names the
Ewald solver but does not print it):

  A_ij = k_e { sum_t' [erfc(alpha r) - erfc(eta_ee r)]/r          (real space)
             + sum_{k in K+} 2 W(k) cos(k.(R_i - R_j)) - pi/(V alpha^2)
             + delta_ij (sqrt(2) eta - 2 alpha)/sqrt(pi)            (self)
             + dipole term }
  b_i  = -k_e { sum_j q_j sum_t [erfc(alpha r) - erfc(eta r)]/r
             + sum_{K+} 2 W(k) sum_j q_j cos(k.(R_i - r_j)) + dipole cross term }

with W(k) = (4 pi / V) exp(-k^2 / 4 alpha^2) / k^2, K+ the half space of
non-zero reciprocal vectors with |k| <= k_c, k_c = 2 alpha sqrt(ln(1/eps_k)),
and the real-space sum over all periodic images t with 0 < r < r_c (t = 0
left out only for i = j).  Units: A, e, V; k_e = 14.399645478425668 V A/e.
All arithmetic is FP64; nothing here is blocked or reordered beyond chunking
sums over k or over rows to bound memory.
"""
from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np
from scipy.special import erf, erfc
import scipy.linalg

KE = 14.399645478425668          # e / (4 pi eps0) in V*A/e (CODATA 2018)
EPS0 = 1.0 / (4.0 * math.pi * KE)  # e / (V*A)

GEOMETRIES = ("slab", "wire", "vacuum3d", "tinfoil", "isolated")


@dataclass
class Params:
    """Ewald cell and method knobs.

    Lx, Ly, Lz: periodic cell (for a slab Lz = slab_factor * h).
    geometry: "slab" (EW3DC in z), "wire" (periodic in z only, Eq. 11),
    "vacuum3d" (3D periodic, spherical vacuum boundary), "tinfoil" (3D
    periodic, no dipole term) or "isolated" (no periodicity at all).
    """
    Lx: float
    Ly: float
    Lz: float
    eta: float = 1.979
    alpha: float = 0.3
    rcut: float = 12.0
    kspace_eps: float = 1e-8
    kcut: float = 0.0
    geometry: str = "slab"

    @property
    def volume(self) -> float:
        return self.Lx * self.Ly * self.Lz

    @property
    def k_cut(self) -> float:
        if self.kcut > 0:
            return self.kcut
        return 2.0 * self.alpha * math.sqrt(math.log(1.0 / self.kspace_eps))


def params_for(w, **over) -> Params:
    """Params of a generated workload (slab cell Lz = slab_factor * h)."""
    p = Params(w.Lx, w.Ly, w.slab_factor * w.h, w.eta, w.alpha, w.rcut, w.kspace_eps)
    for k, v in over.items():
        setattr(p, k, v)
    return p


# ----------------------------------------------------------------------------
# Ewald ingredients
# ----------------------------------------------------------------------------

def kvectors(p: Params):
    """Half-space K+ of reciprocal vectors k = 2 pi (nx/Lx, ny/Ly, nz/Lz),
    |k| <= k_c, one of each +-k pair (nx > 0, or nx = 0 and ny > 0, or
    nx = ny = 0 and nz > 0).  Returns (n (Nk,3) int, k (Nk,3), W (Nk,))."""
    kc = p.k_cut
    nmax = [int(math.floor(kc * L / (2 * math.pi))) for L in (p.Lx, p.Ly, p.Lz)]
    nx = np.arange(0, nmax[0] + 1)
    ny = np.arange(-nmax[1], nmax[1] + 1)
    nz = np.arange(-nmax[2], nmax[2] + 1)
    g = np.stack(np.meshgrid(nx, ny, nz, indexing="ij"), -1).reshape(-1, 3)
    half = (g[:, 0] > 0) | ((g[:, 0] == 0) & (g[:, 1] > 0)) | \
           ((g[:, 0] == 0) & (g[:, 1] == 0) & (g[:, 2] > 0))
    g = g[half]
    k = 2 * math.pi * g / np.array([p.Lx, p.Ly, p.Lz])
    k2 = (k * k).sum(1)
    keep = k2 <= kc * kc
    g, k, k2 = g[keep], k[keep], k2[keep]
    W = (4 * math.pi / p.volume) * np.exp(-k2 / (4 * p.alpha ** 2)) / k2
    return g, k, W


def image_shifts(p: Params, A: np.ndarray, B: np.ndarray):
    """All lattice translations t for which some pair (a in A, b in B) has
    |a - b + t| < r_c.  A translation is kept if the box of differences a - b,
    moved by t, comes within r_c of the origin (exact pruning, no pair is lost)."""
    lo = A.min(0) - B.max(0)
    hi = A.max(0) - B.min(0)
    L = np.array([p.Lx, p.Ly, p.Lz])
    periodic = {"slab": (1, 1, 1), "wire": (1, 1, 1), "vacuum3d": (1, 1, 1),
                "tinfoil": (1, 1, 1), "isolated": (0, 0, 0)}[p.geometry]
    rng = []
    for ax in range(3):
        if not periodic[ax]:
            rng.append([0])
            continue
        nmax = int(math.ceil((p.rcut + max(abs(lo[ax]), abs(hi[ax]))) / L[ax])) + 1
        rng.append(list(range(-nmax, nmax + 1)))
    out = []
    for a in rng[0]:
        for b in rng[1]:
            for c in rng[2]:
                t = np.array([a, b, c]) * L
                # distance from the origin to the box [lo + t, hi + t]
                gap = np.maximum(0.0, np.maximum(lo + t, -(hi + t)))
                if math.sqrt((gap * gap).sum()) < p.rcut:
                    out.append(t)
    return np.array(out).reshape(-1, 3)


def dipole_terms(p: Params):
    """The dipole energy of each geometry as k_e * sum over (c, axis) of
    c * M_axis^2: (2 pi/V) M_z^2 for the slab (Eq. 10), (pi/V)(M_x^2 + M_y^2)
    for the wire (Eq. 11), (2 pi/3V)|M|^2 for a 3D cell in vacuum (spherical
    summation order); none for tin-foil or isolated systems."""
    V = p.volume
    if p.geometry == "slab":
        return [(2 * math.pi / V, 2)]
    if p.geometry == "wire":
        return [(math.pi / V, 0), (math.pi / V, 1)]
    if p.geometry == "vacuum3d":
        c = 2 * math.pi / (3 * V)
        return [(c, 0), (c, 1), (c, 2)]
    return []


# ----------------------------------------------------------------------------
# A: elastance matrix (Eq. 2)
# ----------------------------------------------------------------------------

def elastance(R: np.ndarray, p: Params, rows=None, diag_extra=None) -> np.ndarray:
    """Rows `rows` (default all) of the n x n elastance matrix A (V/e)."""
    R = np.asarray(R, np.float64)
    n = len(R)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    eta_ee = p.eta / math.sqrt(2.0)
    out = np.zeros((len(rows), n))
    Ri = R[rows]

    if p.geometry == "isolated":
        d = Ri[:, None, :] - R[None, :, :]
        r = np.sqrt((d * d).sum(-1))
        same = rows[:, None] == np.arange(n)[None, :]
        rs = np.where(same, 1.0, r)
        out = np.where(same, p.eta * math.sqrt(2.0 / math.pi), erf(eta_ee * rs) / rs)
        out = KE * out
        if diag_extra is not None:
            out[np.arange(len(rows)), rows] += diag_extra[rows]
        return out

    # real space: sum over images t of [erfc(alpha r) - erfc(eta_ee r)]/r, r < r_c
    for t in image_shifts(p, Ri, R):
        d = Ri[:, None, :] - R[None, :, :] + t
        r = np.sqrt((d * d).sum(-1))
        m = (r < p.rcut) & (r > 0.0)
        rs = np.where(m, r, 1.0)
        out += np.where(m, (erfc(p.alpha * rs) - erfc(eta_ee * rs)) / rs, 0.0)

    # k space: sum_{K+} 2 W(k) cos(k.(R_i - R_j)) = C diag(2W) C^T + S diag(2W) S^T
    _, kv, W = kvectors(p)
    for k0 in range(0, len(W), 4096):
        kk, ww = kv[k0:k0 + 4096], 2.0 * W[k0:k0 + 4096]
        ph_all = R @ kk.T
        ph_row = Ri @ kk.T
        out += (np.cos(ph_row) * ww) @ np.cos(ph_all).T + (np.sin(ph_row) * ww) @ np.sin(ph_all).T
    out -= math.pi / (p.volume * p.alpha ** 2)

    # self term on the diagonal
    out[np.arange(len(rows)), rows] += (math.sqrt(2.0) * p.eta - 2.0 * p.alpha) / math.sqrt(math.pi)

    # electrode part of the dipole correction (first term of Eq. 12)
    for c, ax in dipole_terms(p):
        out += 2.0 * c * np.outer(Ri[:, ax], R[:, ax])

    out = KE * out
    if diag_extra is not None:
        out[np.arange(len(rows)), rows] += np.asarray(diag_extra)[rows]
    return out


# ----------------------------------------------------------------------------
# b: electrolyte vector (Eq. 2, Eq. 12 cross term)
# ----------------------------------------------------------------------------

def check_neutral(q: np.ndarray):
    q = np.asarray(q, np.float64)
    if len(q) and abs(q.sum()) > 1e-10 * max(np.abs(q).sum(), 1e-300):
        raise ValueError("electrolyte is not charge neutral")


def structure_factor(r: np.ndarray, q: np.ndarray, kv: np.ndarray) -> np.ndarray:
    """S(k) = sum_j q_j exp(i k.r_j) for every k in kv (complex).  The k set
    is walked in chunks sized to bound memory; each S(k) is one sum over the
    charges whatever the chunk."""
    out = np.zeros(len(kv), np.complex128)
    step = max(16, min(2048, (1 << 22) // max(len(r), 1)))
    for k0 in range(0, len(kv), step):
        ph = r @ kv[k0:k0 + step].T
        out[k0:k0 + step] = (q[:, None] * np.cos(ph)).sum(0) + 1j * (q[:, None] * np.sin(ph)).sum(0)
    return out


def electrolyte_potential(R: np.ndarray, r: np.ndarray, q: np.ndarray, p: Params, rows=None):
    """Potential (V) of the electrolyte point charges at the Gaussian electrode
    atoms `rows` (default all): Ewald real + k space + dipole cross term."""
    R = np.asarray(R, np.float64)
    r = np.asarray(r, np.float64)
    q = np.asarray(q, np.float64)
    check_neutral(q)
    rows = np.arange(len(R)) if rows is None else np.asarray(rows)
    Ri = R[rows]
    phi = np.zeros(len(rows))
    if len(q) == 0:
        return phi
    if p.geometry == "isolated":
        d = Ri[:, None, :] - r[None, :, :]
        rr = np.sqrt((d * d).sum(-1))
        return KE * (erf(p.eta * rr) / rr) @ q

    for t in image_shifts(p, Ri, r):
        for i0 in range(0, len(rows), 512):
            d = Ri[i0:i0 + 512, None, :] - r[None, :, :] + t
            rr = np.sqrt((d * d).sum(-1))
            m = rr < p.rcut
            rs = np.where(m, rr, 1.0)
            phi[i0:i0 + 512] += np.where(m, (erfc(p.alpha * rs) - erfc(p.eta * rs)) / rs, 0.0) @ q

    _, kv, W = kvectors(p)
    Sk = structure_factor(r, q, kv)
    for k0 in range(0, len(W), 4096):
        ph = Ri @ kv[k0:k0 + 4096].T
        w2 = 2.0 * W[k0:k0 + 4096]
        phi += np.cos(ph) @ (w2 * Sk.real[k0:k0 + 4096]) + np.sin(ph) @ (w2 * Sk.imag[k0:k0 + 4096])
    # (the background term -pi/(V alpha^2) sum_j q_j vanishes: neutral electrolyte)

    # electrolyte-electrode dipole cross term (second term of Eq. 12)
    for c, ax in dipole_terms(p):
        M = float(q @ r[:, ax])
        phi += 2.0 * c * Ri[:, ax] * M
    return KE * phi


def potential_vector(R, r, q, p: Params, rows=None) -> np.ndarray:
    """b = -(electrolyte potential at the electrode atoms), so that A q = b + v
    holds at the energy minimum of Eq. 2."""
    return -electrolyte_potential(R, r, q, p, rows)


# ----------------------------------------------------------------------------
# Inversion, neutrality projection, charges (Eqs. 3, 4, 6)
# ----------------------------------------------------------------------------

@dataclass
class Capacitance:
    Ainv: np.ndarray    # A^-1
    u: np.ndarray       # A^-1 e
    s: float            # e^T A^-1 e
    S: np.ndarray       # A^-1 - u u^T / s  (Eq. 4)


def capacitance(A: np.ndarray) -> Capacitance:
    """Cholesky factorisation A = L L^T, A^-1, and the charge-neutral S of Eq. 4.
    Raises numpy.linalg.LinAlgError if A is not positive definite."""
    A = np.asarray(A, np.float64)
    c = scipy.linalg.cho_factor(A, lower=True, check_finite=True)
    Ainv = scipy.linalg.cho_solve(c, np.eye(len(A)))
    Ainv = 0.5 * (Ainv + Ainv.T)
    u = Ainv @ np.ones(len(A))
    s = float(u.sum())
    S = Ainv - np.outer(u, u) / s
    return Capacitance(Ainv, u, s, S)


def applied_potential(eid: np.ndarray, v_electrode) -> np.ndarray:
    """v = G v~ (Eq. 5): each atom gets the potential of its electrode."""
    return np.asarray(v_electrode, np.float64)[np.asarray(eid)]


def charges(S: np.ndarray, b: np.ndarray, v: np.ndarray) -> np.ndarray:
    """q = S (b + v) (Eqs. 4, 6)."""
    return S @ (np.asarray(b, np.float64) + np.asarray(v, np.float64))


def electrode_totals(q: np.ndarray, eid: np.ndarray, n_e: int) -> np.ndarray:
    """Q~ = G^T q (Eq. 7, left-hand side)."""
    out = np.zeros(n_e)
    np.add.at(out, np.asarray(eid), q)
    return out


def electrode_capacitance(S: np.ndarray, eid: np.ndarray, n_e: int) -> np.ndarray:
    """C~ = G^T S G, the electrode-wise capacitance matrix (e/V)."""
    G = np.zeros((len(eid), n_e))
    G[np.arange(len(eid)), eid] = 1.0
    return G.T @ S @ G


def constrained_charges(Ainv: np.ndarray, eid: np.ndarray, n_e: int, b: np.ndarray,
                        Q_target) -> tuple:
    """Constrained charge method (Sec. II.C, Eq. 7): with q = A^-1 (b + G v~),
    G^T q = G^T A^-1 b + G^T A^-1 G v~ = q~_b + C~ v~; solve C~ v~ = Q - q~_b and
    return (q, v~).  The targets must sum to zero (the slab correction and the
    neutral electrolyte need a neutral system)."""
    Q = np.asarray(Q_target, np.float64)
    if abs(Q.sum()) > 1e-12 * max(np.abs(Q).sum(), 1e-300):
        raise ValueError("electrode charge targets must sum to zero")
    G = np.zeros((len(eid), n_e))
    G[np.arange(len(eid)), np.asarray(eid)] = 1.0
    y = Ainv @ np.asarray(b, np.float64)
    Ct = G.T @ Ainv @ G
    vt = np.linalg.solve(Ct, Q - G.T @ y)
    return y + Ainv @ (G @ vt), vt


def finite_field_zeta(z, eid, Lz: float, bottom: int = 0) -> np.ndarray:
    """zeta of the finite-field method (Sec. II.F, Eqs. 13-14): the
    normalised z position z / Lz of every electrode atom, plus one for the
    atoms of the bottom electrode (the offset that makes the cell symmetric
    along z, so that the two electrodes meet across the periodic boundary as
    one conductor).  The field enters as the applied potential v = -dv0 zeta."""
    return np.asarray(z, np.float64) / Lz + (np.asarray(eid) == bottom)


def energy(A, b, v, q) -> float:
    """U_elec of Eq. 2 (eV)."""
    return 0.5 * q @ A @ q - b @ q - v @ q


# ----------------------------------------------------------------------------
# whole pipeline
# ----------------------------------------------------------------------------

@dataclass
class Solution:
    A: np.ndarray
    cap: Capacitance
    b: np.ndarray
    v: np.ndarray
    q: np.ndarray
    Q: np.ndarray


def solve(R, eid, r, q_elyt, p: Params, v_electrode, diag_extra=None) -> Solution:
    """A, S, b, q and the electrode totals for one electrolyte configuration."""
    eid = np.asarray(eid)
    n_e = int(eid.max()) + 1
    A = elastance(R, p, diag_extra=diag_extra)
    cap = capacitance(A)
    b = potential_vector(R, r, q_elyt, p)
    v = applied_potential(eid, v_electrode)
    q = charges(cap.S, b, v)
    return Solution(A, cap, b, v, q, electrode_totals(q, eid, n_e))
