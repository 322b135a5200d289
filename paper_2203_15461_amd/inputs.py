"""Seeded synthetic capacitor inputs.

This module builds coordinates and charges only: graphite electrode layers,
an SPC/E-like water + ion electrolyte between them, and Gaussian-jittered
snapshots of that electrolyte.  It holds none of the constant-potential
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

The paper's own workload (a gold/NaCl capacitor, Sec. III.A and the
simulation-details section of the supplement) is not reproducible here; these
graphite capacitors stand in for it.  Conventions:

* graphene C-C bond d = 1.42 A.  The rectangular 4-atom cell has a zigzag
  period sqrt(3) d and an armchair period 3 d.  Layers of one electrode are
  AB (Bernal) stacked: odd layers are shifted by d along the armchair axis.
* electrode id 0 is the bottom electrode, id 1 the top one.  The applied
  potential is -dV/2 on the bottom and +dV/2 on the top.
* electrolyte sites are kept >= `wall_gap` (3 A) from the inner electrode
  layers; x and y are wrapped into [0, L).
* base seed 15461; snapshot s is drawn with seed 15461 + 1 + s.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

D_CC = 1.42                 # A, graphene bond length
LAYER_SPACING = 3.35        # A, graphite interlayer distance
BASE_SEED = 15461
Q_O, Q_H = -0.8476, 0.4238  # SPC/E-like site charges (e)
R_OH = 1.0                  # A
THETA_HOH = 109.47          # degrees


@dataclass
class Workload:
    """A capacitor: electrode atoms, electrode ids, electrolyte, cell and knobs."""
    name: str
    electrode_xyz: np.ndarray          # (n, 3) float64
    electrode_id: np.ndarray           # (n,) int32, 0 = bottom, 1 = top
    electrolyte_xyz: np.ndarray        # (m, 3) float64
    electrolyte_q: np.ndarray          # (m,) float64, sums to 0
    Lx: float
    Ly: float
    h: float                           # z_top - z_bot of the outermost layers
    delta_v: float                     # V, top minus bottom
    eta: float = 1.979
    alpha: float = 0.3
    rcut: float = 12.0
    kspace_eps: float = 1e-8
    slab_factor: float = 3.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.electrode_xyz.shape[0])

    @property
    def m(self) -> int:
        return int(self.electrolyte_xyz.shape[0])

    @property
    def v_electrode(self) -> np.ndarray:
        """Per-electrode applied potential (V): bottom -dV/2, top +dV/2."""
        return np.array([-0.5 * self.delta_v, 0.5 * self.delta_v])

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def graphene_layer(n_x: int, n_y: int, x_axis: str = "zigzag", shifted: bool = False,
                   dcc: float = D_CC):
    """One rectangular graphene sheet of n_x * n_y 4-atom cells.

    `x_axis` names which lattice period runs along x ("zigzag": sqrt(3) d,
    "armchair": 3 d).  `shifted` moves the sheet by d along the armchair axis
    (the B layer of AB stacking).  Returns (xy (4 n_x n_y, 2), Lx, Ly).
    """
    pz, pa = math.sqrt(3.0) * dcc, 3.0 * dcc
    # cell coordinates (u along zigzag period, w along armchair period)
    base = np.array([[0.0, 0.0],
                     [0.5 * pz, 0.5 * dcc],
                     [0.5 * pz, 1.5 * dcc],
                     [0.0, 2.0 * dcc]])
    if shifted:
        base[:, 1] += dcc
    if x_axis == "zigzag":
        nu, nw = n_x, n_y
    elif x_axis == "armchair":
        nu, nw = n_y, n_x
    else:
        raise ValueError(x_axis)
    iu, iw = np.meshgrid(np.arange(nu), np.arange(nw), indexing="ij")
    cells = np.stack([iu.ravel() * pz, iw.ravel() * pa], axis=1)
    uw = (cells[:, None, :] + base[None, :, :]).reshape(-1, 2)
    Lu, Lw = nu * pz, nw * pa
    uw[:, 1] = np.mod(uw[:, 1], Lw)
    if x_axis == "zigzag":
        return uw, Lu, Lw
    return uw[:, ::-1].copy(), Lw, Lu


def electrode_stack(n_x, n_y, z_layers, x_axis="zigzag"):
    """Stack graphene layers at the given z values (AB stacking by layer index)."""
    out = []
    Lx = Ly = None
    for li, z in enumerate(z_layers):
        xy, Lx, Ly = graphene_layer(n_x, n_y, x_axis=x_axis, shifted=bool(li % 2))
        out.append(np.column_stack([xy, np.full(len(xy), float(z))]))
    return np.concatenate(out, axis=0), Lx, Ly


def _random_rotations(rng, k):
    """k uniformly random rotation matrices (normalised 4-normal quaternions)."""
    qv = rng.normal(size=(k, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)


def water_ion_electrolyte(rng, Lx, Ly, z_lo, z_hi, n_water, n_pairs):
    """SPC/E-like rigid waters (random orientation) plus n_pairs of +1/-1 ions.

    Every site lies in [z_lo, z_hi]; oxygens are drawn 1 A inside that range so
    the hydrogens stay inside it too.  Returns (xyz (m, 3), q (m,)).
    """
    th = math.radians(THETA_HOH) / 2.0
    ref = np.array([[0.0, 0.0, 0.0],
                    [R_OH * math.sin(th), 0.0, R_OH * math.cos(th)],
                    [-R_OH * math.sin(th), 0.0, R_OH * math.cos(th)]])
    o = np.column_stack([rng.uniform(0, Lx, n_water), rng.uniform(0, Ly, n_water),
                         rng.uniform(z_lo + R_OH, z_hi - R_OH, n_water)])
    rot = _random_rotations(rng, n_water)
    sites = o[:, None, :] + np.einsum("wij,sj->wsi", rot, ref)
    wq = np.tile([Q_O, Q_H, Q_H], n_water)
    ions = np.column_stack([rng.uniform(0, Lx, 2 * n_pairs), rng.uniform(0, Ly, 2 * n_pairs),
                            rng.uniform(z_lo, z_hi, 2 * n_pairs)])
    iq = np.concatenate([np.ones(n_pairs), -np.ones(n_pairs)])
    xyz = np.concatenate([sites.reshape(-1, 3), ions], axis=0)
    q = np.concatenate([wq, iq])
    xyz[:, 0] = np.mod(xyz[:, 0], Lx)
    xyz[:, 1] = np.mod(xyz[:, 1], Ly)
    return xyz, q


def _two_electrodes(n_x, n_y, z_bot_layers, z_top_layers, x_axis):
    bot, Lx, Ly = electrode_stack(n_x, n_y, z_bot_layers, x_axis)
    top, _, _ = electrode_stack(n_x, n_y, z_top_layers, x_axis)
    xyz = np.concatenate([bot, top], axis=0)
    eid = np.concatenate([np.zeros(len(bot), np.int32), np.ones(len(top), np.int32)])
    return xyz, eid, Lx, Ly


def small_capacitor(variant: str = "a", seed: int = BASE_SEED, n_ions: int = 100) -> Workload:
    """Two single graphene layers at z = 0 and 30 A with 100 +-1 e point charges.

    variant "a": 144 atoms per layer in 14.757 x 25.560 A (6 x 6 cells);
    variant "b": 96 atoms per layer in 14.757 x 17.040 A (6 x 4 cells).
    Ions are uniform in x, y and in z in [3, 27] A.  dV = 1 V.
    """
    n_y = {"a": 6, "b": 4}[variant]
    xyz, eid, Lx, Ly = _two_electrodes(6, n_y, [0.0], [30.0], "zigzag")
    rng = np.random.default_rng(seed)
    half = n_ions // 2
    r = np.column_stack([rng.uniform(0, Lx, n_ions), rng.uniform(0, Ly, n_ions),
                         rng.uniform(3.0, 27.0, n_ions)])
    q = np.concatenate([np.ones(half), -np.ones(n_ions - half)])
    return Workload(f"small_capacitor_{variant}", xyz, eid, r, q, Lx, Ly, 30.0, 1.0)


def graphite_capacitor(n_x: int = 8, n_y: int = 15, gap: float = 50.0, seed: int = BASE_SEED,
                       n_water: int | None = None, n_pairs: int | None = None,
                       wall_gap: float = 3.0, delta_v: float = 2.0, name: str | None = None) -> Workload:
    """Two 3-layer AB graphite electrodes with a water + NaCl electrolyte.

    Defaults: 8 armchair x 15 zigzag cells per layer (480 atoms, 34.080 x
    36.893 A), layers at 0/3.35/6.70 and gap + (6.70, 10.05, 13.40), 2000
    waters and 64 ion pairs (m = 6128), dV = 2 V.
    """
    zb = [0.0, LAYER_SPACING, 2 * LAYER_SPACING]
    zt = [zb[-1] + gap + k * LAYER_SPACING for k in range(3)]
    xyz, eid, Lx, Ly = _two_electrodes(n_x, n_y, zb, zt, "armchair")
    rng = np.random.default_rng(seed)
    if n_water is None:
        n_water = 2000
    if n_pairs is None:
        n_pairs = 64
    r, q = water_ion_electrolyte(rng, Lx, Ly, zb[-1] + wall_gap, zt[0] - wall_gap, n_water, n_pairs)
    return Workload(name or f"graphite_capacitor_{len(xyz)}", xyz, eid, r, q, Lx, Ly,
                    zt[-1] - zb[0], delta_v)


def scaled_graphite_capacitor(n_target: int, seed: int = BASE_SEED) -> Workload:
    """A graphite capacitor with about n_target electrode atoms (6 layers of
    4 n_x n_y atoms, near-square cell), 10 water charges per electrode atom and
    1 M of +-1 e ions in the 50 A gap."""
    cells = max(1, round(n_target / 24))
    # a square cell needs n_y = sqrt(3) n_x (armchair period 3 d along x)
    n_x = max(1, round(math.sqrt(cells / math.sqrt(3.0))))
    n_y = max(1, round(cells / n_x))
    n = 24 * n_x * n_y
    Lx, Ly = n_x * 3 * D_CC, n_y * math.sqrt(3) * D_CC
    n_water = (10 * n) // 3
    vol_l = Lx * Ly * 50.0 * 1e-27          # litres
    n_pairs = max(1, round(1.0 * 6.02214076e23 * vol_l))
    return graphite_capacitor(n_x, n_y, 50.0, seed, n_water, n_pairs,
                              name=f"scaled_graphite_capacitor_{n}")


def snapshot(w: Workload, s: int, sigma: float = 0.1) -> np.ndarray:
    """Electrolyte coordinates of snapshot s: every coordinate jittered by an
    independent N(0, sigma^2) draw (seed BASE_SEED + 1 + s); x, y re-wrapped."""
    rng = np.random.default_rng(BASE_SEED + 1 + s)
    r = w.electrolyte_xyz + rng.normal(0.0, sigma, size=w.electrolyte_xyz.shape)
    r[:, 0] = np.mod(r[:, 0], w.Lx)
    r[:, 1] = np.mod(r[:, 1], w.Ly)
    return r


def snapshots(w: Workload, count: int, start: int = 0, sigma: float = 0.1) -> np.ndarray:
    """(count, m, 3) stack of jittered electrolyte snapshots."""
    return np.stack([snapshot(w, start + s, sigma) for s in range(count)])


def isolated_cluster(n_elec: int, n_ions: int, seed: int = BASE_SEED, spread: float = 4.0):
    """Tiny cluster: n_elec electrode atoms (two electrodes, split in half) and
    n_ions neutral +-1 point charges, all within a `spread`-A box around the
    origin with every pair >= 1.2 A apart.  Returns (R, eid, r, q)."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n_elec + n_ions:
        p = rng.uniform(-spread / 2, spread / 2, 3)
        if all(np.linalg.norm(p - o) >= 1.2 for o in pts):
            pts.append(p)
    pts = np.array(pts)
    R, r = pts[:n_elec], pts[n_elec:]
    eid = np.array([0] * (n_elec // 2) + [1] * (n_elec - n_elec // 2), np.int32)
    q = np.array([1.0 if k % 2 == 0 else -1.0 for k in range(n_ions)])
    if n_ions % 2:
        q[-1] = 0.0
    return R, eid, r, q


def coaxial_tubes(n1: int, n2: int, dcc: float = D_CC):
    """Two co-axial armchair tubes (n1,n1)@(n2,n2), one axial period
    (sqrt(3) d) along z, axis at the origin.  Returns (R, eid, R1, R2, period)."""
    period = math.sqrt(3.0) * dcc
    out, ids, radii = [], [], []
    for e, nn in enumerate((n1, n2)):
        circ = 3.0 * nn * dcc
        rad = circ / (2.0 * math.pi)
        # armchair tube: the armchair period (3 d) runs around the circumference
        xy, _, _ = graphene_layer(nn, 1, x_axis="armchair")   # x: armchair (circumference), y: zigzag (axis)
        phi = xy[:, 0] / rad
        out.append(np.column_stack([rad * np.cos(phi), rad * np.sin(phi), xy[:, 1]]))
        ids.append(np.full(len(xy), e, np.int32))
        radii.append(rad)
    return np.concatenate(out), np.concatenate(ids), radii[0], radii[1], period
