"""Seeded scene descriptors (inputs only).

Every generator returns an `EnvDesc` whose float arrays hold float32-representable
values, so the FP64 oracle and the FP32 GPU path start from bit-identical inputs.
Units are SI, z is up, quaternions are (w, x, y, z), angular velocities are in the
world frame.

Body conventions used by the descriptors:
  * a rigid body with mass 0 is static (an obstacle: infinite mass, never moves);
  * particles get their mass from the tetrahedra that use them plus an optional
    explicit `particle_mass` (used by the tiny closed-form cases);
  * box shapes carry half-extents; capsules carry (radius, half-length, 0) with the
    segment along the body x axis; SHAPE_NONE bodies have no collision geometry;
  * joints connect body A (index or -1 = world) to body B; anchors, axes and
    reference (perpendicular) directions are given in each body's own frame.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

SHAPE_BOX, SHAPE_CAPSULE, SHAPE_NONE = 0, 1, 2
JOINT_REVOLUTE, JOINT_PRISMATIC = 0, 1
NCP_FB, NCP_MIN = 0, 1
RMODE_IDENTITY, RMODE_H2, RMODE_H2_EFFMASS = 0, 1, 2
FEM_FULL_PROJECTED, FEM_DIAGONAL = 0, 1
WARM_ZERO, WARM_PREV, WARM_LEARNED, WARM_HYBRID = 0, 1, 2, 3
TET_NEOHOOKEAN, TET_LINEAR = 0, 1


def round_to_f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclasses.dataclass
class SolverParams:
    ncp: int = NCP_FB
    rmode: int = RMODE_H2_EFFMASS
    damping: float = 0.75          # constant Newton step fraction t
    eps: float = 1e-6              # Schur-matrix regularisation
    geo_stiff: int = 1             # diagonal geometric stiffness on particle DOFs
    fem_mode: int = FEM_FULL_PROJECTED
    margin: float = 5e-3           # contact creation distance
    warm: int = WARM_ZERO
    line_search: int = 0           # 1: back-tracking on the L2 merit (frictionless scenes)
    linear: int = 0                # 0 PCR (the method), 1 PCG (comparison solver)
    islands: int = 0               # 1: independent PCR scalars per island of an env
    watchdog: int = 0              # 1: return the step's lowest-merit iterate when the merit
                                   # blows up (a safeguard Sec. 8.1 names); 0: the paper's method


@dataclasses.dataclass
class EnvDesc:
    rigid_mass: np.ndarray
    rigid_inertia: np.ndarray
    rigid_x: np.ndarray
    rigid_q: np.ndarray
    rigid_v: np.ndarray
    rigid_w: np.ndarray
    rigid_shape: np.ndarray
    rigid_extent: np.ndarray
    particle_x: np.ndarray
    particle_v: np.ndarray
    particle_rest: np.ndarray
    particle_mass: np.ndarray
    tet_ids: np.ndarray
    tet_material: np.ndarray
    joint_type: np.ndarray
    joint_body: np.ndarray
    joint_anchor: np.ndarray
    joint_axis: np.ndarray
    joint_ref: np.ndarray
    joint_drive: np.ndarray
    mu: float = 0.5
    gravity: tuple = (0.0, 0.0, -9.81)
    ground: int = 1
    max_contacts: int = 256
    tet_model: int = 0   # TET_NEOHOOKEAN (3 rows per tet) or TET_LINEAR (6 rows per tet)
    name: str = ""

    @property
    def n_rigid(self):
        return int(self.rigid_mass.shape[0])

    @property
    def n_particles(self):
        return int(self.particle_x.shape[0])

    @property
    def n_tets(self):
        return int(self.tet_ids.shape[0])

    @property
    def n_joints(self):
        return int(self.joint_type.shape[0])

    def finalize(self):
        """Coerce dtypes/shapes and round floats to float32-representable values."""
        f = lambda a, shape: round_to_f32(np.asarray(a, dtype=np.float64).reshape(shape))
        nr, npart, nt, nj = (len(self.rigid_mass), len(self.particle_x),
                             len(self.tet_ids), len(self.joint_type))
        self.rigid_mass = f(self.rigid_mass, (nr,))
        self.rigid_inertia = f(self.rigid_inertia, (nr, 3))
        self.rigid_x = f(self.rigid_x, (nr, 3))
        q = np.asarray(self.rigid_q, dtype=np.float64).reshape(nr, 4)
        if nr:
            q = q / np.linalg.norm(q, axis=1, keepdims=True)
        self.rigid_q = round_to_f32(q)
        self.rigid_v = f(self.rigid_v, (nr, 3))
        self.rigid_w = f(self.rigid_w, (nr, 3))
        self.rigid_shape = np.asarray(self.rigid_shape, dtype=np.int32).reshape(nr)
        self.rigid_extent = f(self.rigid_extent, (nr, 3))
        self.particle_x = f(self.particle_x, (npart, 3))
        self.particle_v = f(self.particle_v, (npart, 3))
        self.particle_rest = f(self.particle_rest, (npart, 3))
        self.particle_mass = f(self.particle_mass, (npart,))
        self.tet_ids = np.ascontiguousarray(np.asarray(self.tet_ids, dtype=np.int32).reshape(nt, 4))
        self.tet_material = f(self.tet_material, (nt, 3))
        self.joint_type = np.asarray(self.joint_type, dtype=np.int32).reshape(nj)
        self.joint_body = np.ascontiguousarray(np.asarray(self.joint_body, dtype=np.int32).reshape(nj, 2))
        self.joint_anchor = f(self.joint_anchor, (nj, 2, 3))
        self.joint_axis = f(self.joint_axis, (nj, 2, 3))
        self.joint_ref = f(self.joint_ref, (nj, 2, 3))
        self.joint_drive = f(self.joint_drive, (nj, 6))
        self.mu = float(np.float32(self.mu))
        self.gravity = tuple(float(np.float32(g)) for g in self.gravity)
        self.ground = int(self.ground)
        self.max_contacts = int(self.max_contacts)
        self.tet_model = int(self.tet_model)
        return self

    def rows_estimate(self):
        return 6 * self.n_joints + 3 * self.max_contacts + self.tet_rows * self.n_tets

    @property
    def tet_rows(self):
        return 6 if self.tet_model == TET_LINEAR else 3


# ----------------------------------------------------------------------------
# helpers (inputs: physical properties of shapes, meshes, frames)
# ----------------------------------------------------------------------------

def box_inertia(mass, half):
    a, b, c = half
    return np.array([mass / 3.0 * (b * b + c * c),
                     mass / 3.0 * (a * a + c * c),
                     mass / 3.0 * (a * a + b * b)])


def capsule_inertia(mass, radius, half_len):
    """Solid cylinder of length 2*half_len + radius caps lumped into it (input only)."""
    L = 2.0 * half_len + radius
    ix = 0.5 * mass * radius * radius
    iyz = mass * (3.0 * radius * radius + L * L) / 12.0
    return np.array([ix, iyz, iyz])


def quat_from_axis_angle(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    s = math.sin(0.5 * angle)
    return np.array([math.cos(0.5 * angle), axis[0] * s, axis[1] * s, axis[2] * s])


def _empty(n_rigid=0, n_particles=0, n_tets=0, n_joints=0, **kw) -> EnvDesc:
    d = EnvDesc(
        rigid_mass=np.zeros(n_rigid), rigid_inertia=np.zeros((n_rigid, 3)),
        rigid_x=np.zeros((n_rigid, 3)), rigid_q=np.tile([1.0, 0, 0, 0], (n_rigid, 1)),
        rigid_v=np.zeros((n_rigid, 3)), rigid_w=np.zeros((n_rigid, 3)),
        rigid_shape=np.zeros(n_rigid, np.int32), rigid_extent=np.zeros((n_rigid, 3)),
        particle_x=np.zeros((n_particles, 3)), particle_v=np.zeros((n_particles, 3)),
        particle_rest=np.zeros((n_particles, 3)), particle_mass=np.zeros(n_particles),
        tet_ids=np.zeros((n_tets, 4), np.int32), tet_material=np.zeros((n_tets, 3)),
        joint_type=np.zeros(n_joints, np.int32), joint_body=np.zeros((n_joints, 2), np.int32),
        joint_anchor=np.zeros((n_joints, 2, 3)), joint_axis=np.zeros((n_joints, 2, 3)),
        joint_ref=np.zeros((n_joints, 2, 3)), joint_drive=np.zeros((n_joints, 6)))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _concat_rigid(bodies):
    """bodies: list of dicts(mass, inertia, x, q, v, w, shape, extent)."""
    keys = ["mass", "inertia", "x", "q", "v", "w", "shape", "extent"]
    out = {}
    for k in keys:
        out[k] = np.array([b[k] for b in bodies]) if bodies else np.zeros((0,))
    return out


def _box(mass, half, x, q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0)):
    half = np.asarray(half, dtype=np.float64)
    return dict(mass=mass, inertia=box_inertia(mass, half) if mass > 0 else np.zeros(3),
                x=np.asarray(x, np.float64), q=np.asarray(q, np.float64),
                v=np.asarray(v, np.float64), w=np.asarray(w, np.float64),
                shape=SHAPE_BOX, extent=half)


def _nocollide(b):
    b = dict(b)
    b["shape"] = SHAPE_NONE
    return b


def _capsule(mass, radius, half_len, x, q=(1, 0, 0, 0)):
    return dict(mass=mass, inertia=capsule_inertia(mass, radius, half_len),
                x=np.asarray(x, np.float64), q=np.asarray(q, np.float64),
                v=np.zeros(3), w=np.zeros(3), shape=SHAPE_CAPSULE,
                extent=np.array([radius, half_len, 0.0]))


def _set_rigid(d: EnvDesc, bodies):
    if not bodies:
        return
    r = _concat_rigid(bodies)
    d.rigid_mass = r["mass"].astype(np.float64)
    d.rigid_inertia = r["inertia"].reshape(-1, 3)
    d.rigid_x = r["x"].reshape(-1, 3)
    d.rigid_q = r["q"].reshape(-1, 4)
    d.rigid_v = r["v"].reshape(-1, 3)
    d.rigid_w = r["w"].reshape(-1, 3)
    d.rigid_shape = r["shape"].astype(np.int32)
    d.rigid_extent = r["extent"].reshape(-1, 3)


def _orient_tets(x, tets):
    """Swap two ids of negatively oriented tets (mesh hygiene, input side)."""
    a = x[tets[:, 1]] - x[tets[:, 0]]
    b = x[tets[:, 2]] - x[tets[:, 0]]
    c = x[tets[:, 3]] - x[tets[:, 0]]
    vol = np.einsum("ij,ij->i", np.cross(a, b), c)
    neg = vol < 0
    t = tets.copy()
    t[neg, 2], t[neg, 3] = tets[neg, 3], tets[neg, 2]
    return t


# 5-tet split of a hex; corners numbered by bits (x=1, y=2, z=4).
_HEX_EVEN = [(0, 1, 2, 4), (3, 1, 7, 2), (5, 1, 4, 7), (6, 2, 7, 4), (1, 2, 4, 7)]
_HEX_ODD = [(1, 0, 3, 5), (2, 0, 6, 3), (4, 0, 5, 6), (7, 3, 5, 6), (0, 3, 5, 6)]


def hex_grid_tets(nx, ny, nz, cell, origin=(0.0, 0.0, 0.0), keep=None):
    """Regular hex grid split into 5 tets per cell with alternating mirror by cell
    parity (conforming).  `keep(i,j,k)` optionally selects cells.  Returns
    (particle positions [np,3], tet ids [nt,4]) with unused corners dropped."""
    origin = np.asarray(origin, dtype=np.float64)
    vid = -np.ones((nx + 1, ny + 1, nz + 1), dtype=np.int64)
    tets = []
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if keep is not None and not keep(i, j, k):
                    continue
                cells.append((i, j, k))
    for (i, j, k) in cells:
        for c in range(8):
            ci, cj, ck = i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)
            if vid[ci, cj, ck] < 0:
                vid[ci, cj, ck] = 0  # mark used
    used = np.argwhere(vid >= 0)
    # deterministic numbering: x fastest, then y, then z
    order = np.lexsort((used[:, 0], used[:, 1], used[:, 2]))
    used = used[order]
    for n, (ci, cj, ck) in enumerate(used):
        vid[ci, cj, ck] = n
    x = origin[None, :] + used.astype(np.float64) * cell
    for (i, j, k) in cells:
        corner = [vid[i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)] for c in range(8)]
        pattern = _HEX_EVEN if (i + j + k) % 2 == 0 else _HEX_ODD
        for t in pattern:
            tets.append([corner[t[0]], corner[t[1]], corner[t[2]], corner[t[3]]])
    tets = np.asarray(tets, dtype=np.int64).reshape(-1, 4)
    if len(tets):
        tets = _orient_tets(x, tets)
    return x, tets.astype(np.int32)


def sphere_tets(radius, cell, center):
    n = int(math.ceil(2 * radius / cell))
    origin = np.asarray(center, np.float64) - 0.5 * n * cell

    def keep(i, j, k):
        c = origin + (np.array([i, j, k]) + 0.5) * cell
        return np.linalg.norm(c - np.asarray(center)) <= radius

    return hex_grid_tets(n, n, n, cell, origin=origin, keep=keep)


def _set_tets(d: EnvDesc, x, tets, E, nu, rho, v=None):
    d.particle_x = x
    d.particle_rest = x.copy()
    d.particle_v = np.zeros_like(x) if v is None else v
    d.particle_mass = np.zeros(len(x))
    d.tet_ids = tets
    d.tet_material = np.tile([E, nu, rho], (len(tets), 1))


def _revolute(a, b, anchor_a, anchor_b, axis_a, axis_b, ref_a, ref_b, drive=(0, 0, 0, 0, 0, 0)):
    return dict(type=JOINT_REVOLUTE, body=(a, b), anchor=(anchor_a, anchor_b),
                axis=(axis_a, axis_b), ref=(ref_a, ref_b), drive=drive)


def _prismatic(a, b, anchor_a, anchor_b, axis_a, axis_b, ref_a, ref_b, drive=(0, 0, 0, 0, 0, 0)):
    return dict(type=JOINT_PRISMATIC, body=(a, b), anchor=(anchor_a, anchor_b),
                axis=(axis_a, axis_b), ref=(ref_a, ref_b), drive=drive)


def _set_joints(d: EnvDesc, joints):
    nj = len(joints)
    d.joint_type = np.array([j["type"] for j in joints], np.int32).reshape(nj)
    d.joint_body = np.array([j["body"] for j in joints], np.int32).reshape(nj, 2)
    d.joint_anchor = np.array([j["anchor"] for j in joints], np.float64).reshape(nj, 2, 3)
    d.joint_axis = np.array([j["axis"] for j in joints], np.float64).reshape(nj, 2, 3)
    d.joint_ref = np.array([j["ref"] for j in joints], np.float64).reshape(nj, 2, 3)
    d.joint_drive = np.array([j["drive"] for j in joints], np.float64).reshape(nj, 6)


# ----------------------------------------------------------------------------
# benchmark workloads
# ----------------------------------------------------------------------------

def cube_stack(seed=0, n=8, side=0.1, mass=1.0, mu=0.5, jitter=1e-3):
    """Stack of `n` rigid cubes on the ground with seeded xy jitter."""
    rng = np.random.default_rng(seed)
    half = 0.5 * side
    bodies = []
    for k in range(n):
        j = rng.uniform(-jitter, jitter, size=2)
        bodies.append(_box(mass, (half, half, half), (j[0], j[1], half + side * k)))
    d = _empty(mu=mu, max_contacts=128, name=f"cube_stack(seed={seed})")
    _set_rigid(d, bodies)
    return d.finalize()


def stretched_sheet(speed=0.5, nx=8, ny=4, cell=0.05, E=1e5, nu=0.45, rho=1000.0):
    """A neo-Hookean sheet (nx x ny x 1 hexes, 5 tets each) pulled apart in x: the
    particles of both end columns are made heavy (1e6 kg) and given opposite x
    velocities, so they move almost kinematically and the strain grows by about
    2 speed h / (nx cell) per step.  No gravity, no ground (the paper's material
    extension / stretched-sheet test)."""
    x, tets = hex_grid_tets(nx, ny, 1, cell, origin=(0.0, 0.0, 0.0))
    d = _empty(mu=0.0, max_contacts=1, name=f"stretched_sheet(speed={speed})")
    _set_tets(d, x, tets, E, nu, rho)
    d.gravity = np.zeros(3)
    d.ground = 0
    px = np.asarray(d.particle_x)[:, 0]
    left, right = px < 0.5 * cell, px > px.max() - 0.5 * cell
    d.particle_mass = np.asarray(d.particle_mass, np.float64).copy()
    d.particle_mass[left | right] = 1e6
    d.particle_v = np.zeros((len(px), 3))
    d.particle_v[left, 0] = -speed
    d.particle_v[right, 0] = speed
    return d.finalize()


def extension_bar(stretch=1.0, tet_model=TET_NEOHOOKEAN, speed=0.0, nx=12, ny=2, nz=2, cell=0.05, E=1e5,
                  nu=0.45, rho=1000.0):
    """A bar of nx x ny x nz hexes (5 tets each) along x, pre-stretched by the factor
    1 + stretch with its cross-section at rest size.  The particles of both end
    sections are heavy (1e6 kg): at rest they hold the length and the interior relaxes;
    with speed > 0 the two ends move apart at that speed each and stretch the bar
    gradually.  No gravity, no ground (the material-extension test: linear against
    hyperelastic volume change, E = 1e5 Pa, nu = 0.45)."""
    x, tets = hex_grid_tets(nx, ny, nz, cell, origin=(0.0, 0.0, 0.0))
    d = _empty(mu=0.0, max_contacts=1, tet_model=tet_model,
               name=f"extension_bar(stretch={stretch},model={tet_model})")
    _set_tets(d, x, tets, E, nu, rho)
    d.particle_x = x * np.array([1.0 + stretch, 1.0, 1.0])
    d.gravity = np.zeros(3)
    d.ground = 0
    px = x[:, 0]
    ends = (px < 0.5 * cell) | (px > px.max() - 0.5 * cell)
    d.particle_mass = np.where(ends, 1e6, 0.0)
    d.particle_v = np.zeros_like(x)
    d.particle_v[px < 0.5 * cell, 0] = -speed
    d.particle_v[px > px.max() - 0.5 * cell, 0] = speed
    return d.finalize()


def heavy_stack(seed=0, n=5, side=0.1, base_mass=8.0, ratio=8.0, mu=0.5, jitter=1e-3):
    """Stack of `n` cubes whose masses grow geometrically upwards, m_k = base * ratio^k
    (the heavy stack of the paper's rigid tests: 8, 64, ..., 32768 kg, 4096:1)."""
    rng = np.random.default_rng(seed)
    half = 0.5 * side
    bodies = []
    for k in range(n):
        j = rng.uniform(-jitter, jitter, size=2)
        bodies.append(_box(base_mass * ratio ** k, (half, half, half), (j[0], j[1], half + side * k)))
    d = _empty(mu=mu, max_contacts=128, name=f"heavy_stack(seed={seed},n={n})")
    _set_rigid(d, bodies)
    return d.finalize()


def tet_block_with_boxes(seed=0, cells=12, side=0.6, n_boxes=16, E=1e5, nu=0.45, rho=1000.0,
                         mu=0.6, max_contacts=2048, tet_model=TET_NEOHOOKEAN):
    """Elastic block (cells^3 hexes, 5 tets each; neo-Hookean unless `tet_model` says
    linear) on the ground with boxes dropped on it."""
    rng = np.random.default_rng(seed)
    cell = side / cells
    x, tets = hex_grid_tets(cells, cells, cells, cell, origin=(-0.5 * side, -0.5 * side, 0.0))
    d = _empty(mu=mu, max_contacts=max_contacts, tet_model=tet_model,
               name=f"tet_block(seed={seed},cells={cells},model={tet_model})")
    _set_tets(d, x, tets, E, nu, rho)
    bodies = []
    for _ in range(n_boxes):
        s = rng.uniform(0.05, 0.15)
        h = 0.5 * s
        px, py = rng.uniform(-0.5 * side + h, 0.5 * side - h, size=2)
        pz = side + h + rng.uniform(0.05, 0.3)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        bodies.append(_box(rho * s ** 3, (h, h, h), (px, py, pz),
                           q=quat_from_axis_angle((0, 0, 1), yaw)))
    _set_rigid(d, bodies)
    return d.finalize()


def batched_env(seed, tets_max=3000, boxes=(5, 40), joints_max=12, max_contacts=1024, tet_model=TET_NEOHOOKEAN):
    """One environment of the uneven batch: a seeded number of boxes (some stacked on
    the ground, some dropped on a tet block, some hinged into chains), 0..joints_max
    revolute joints and 0..tets_max tets (neo-Hookean unless `tet_model` says linear;
    the model does not change the geometry or the random draws)."""
    rng = np.random.default_rng(seed)
    n_boxes = int(rng.integers(boxes[0], boxes[1] + 1))
    n_joints = int(rng.integers(0, joints_max + 1))
    n_tet_target = int(rng.integers(0, tets_max + 1))
    mu = float(rng.uniform(0.3, 1.0))
    d = _empty(mu=mu, max_contacts=max_contacts, tet_model=tet_model, name=f"batched_env(seed={seed})")
    cell = 0.05
    # near-cubic grid with 5*nx*ny*nz <= target
    nhex = n_tet_target // 5
    nx = ny = nz = 0
    if nhex >= 1:
        c = max(1, int(round(nhex ** (1.0 / 3.0))))
        nx = ny = c
        nz = max(1, nhex // (nx * ny))
        while nx * ny * nz > nhex:
            nz -= 1
            if nz == 0:
                nx = ny = max(1, nx - 1)
                nz = max(1, nhex // (nx * ny))
    block_top = 0.0
    if nx * ny * nz >= 1:
        x, tets = hex_grid_tets(nx, ny, nz, cell, origin=(0.0, 0.0, 0.0))
        _set_tets(d, x, tets, 1e5, 0.45, 1000.0)
        block_top = nz * cell
    n_joints = min(n_joints, n_boxes - 1)
    bodies = []
    joints = []
    # hinged chains along x on the ground at y < 0
    n_chain_boxes = n_joints + (1 if n_joints > 0 else 0)
    if n_joints > 0:
        # split into chains of <= 4 boxes
        remaining = n_chain_boxes
        sizes = []
        while remaining > 0:
            k = min(4, remaining)
            if remaining - k == 1:
                k -= 1
            sizes.append(k)
            remaining -= k
        n_joints = sum(s - 1 for s in sizes)
        n_chain_boxes = sum(sizes)
        s, gap = 0.1, 0.02
        h = 0.5 * s
        for ci, k in enumerate(sizes):
            y = -0.4 - 0.3 * ci
            first = len(bodies)
            for b in range(k):
                bodies.append(_box(1000.0 * s ** 3, (h, h, h),
                                   (-0.4 + b * (s + gap), y, h + 0.002)))
            for b in range(k - 1):
                ia, ib = first + b, first + b + 1
                joints.append(_revolute(ia, ib, (h + 0.5 * gap, 0.0, 0.0), (-h - 0.5 * gap, 0.0, 0.0),
                                        (0.0, 1.0, 0.0), (0.0, 1.0, 0.0),
                                        (1.0, 0.0, 0.0), (1.0, 0.0, 0.0)))
    # free boxes: some dropped on the block, the rest stacked on the ground at x < -0.6.
    # Dropped boxes sit in a grid of cells over the block top (pitch 0.22 m: a 0.15 m box
    # turned about z spans up to 0.212 m), at most two layers 0.17 m apart, starting
    # 1-2 cm above the block, so that no two bodies overlap at t = 0.
    n_free = n_boxes - len(bodies)
    on_block = n_free // 3 if block_top > 0 else 0
    lx, ly = nx * cell, ny * cell
    pitch = 0.22
    ncx, ncy = max(1, int(lx // pitch)), max(1, int(ly // pitch))
    on_block = min(on_block, 2 * ncx * ncy)
    for b in range(on_block):
        layer, slot = divmod(b, ncx * ncy)
        i, j = divmod(slot, ncy)
        s = rng.uniform(0.05, 0.15)
        h = 0.5 * s
        px = (i + 0.5) * lx / ncx + rng.uniform(-5e-3, 5e-3)
        py = (j + 0.5) * ly / ncy + rng.uniform(-5e-3, 5e-3)
        pz = block_top + 0.01 + rng.uniform(0.0, 0.01) + h + 0.17 * layer
        bodies.append(_box(1000.0 * s ** 3, (h, h, h), (px, py, pz),
                           q=quat_from_axis_angle((0, 0, 1), rng.uniform(0, 2 * math.pi))))
    rest = n_free - on_block
    stack_id = 0
    while rest > 0:
        height = int(min(rest, rng.integers(1, 4)))
        sx = -0.8 - 0.3 * (stack_id % 4)
        sy = 0.3 * (stack_id // 4)
        z = 0.0
        for _ in range(height):
            s = rng.uniform(0.05, 0.15)
            h = 0.5 * s
            j = rng.uniform(-2e-3, 2e-3, size=2)
            bodies.append(_box(1000.0 * s ** 3, (h, h, h), (sx + j[0], sy + j[1], z + h + 1e-3)))
            z += s + 1e-3
        rest -= height
        stack_id += 1
    _set_rigid(d, bodies)
    _set_joints(d, joints)
    return d.finalize()


def batched_envs(n_envs=4096, base_seed=1000, **kw) -> List[EnvDesc]:
    return [batched_env(base_seed + e, **kw) for e in range(n_envs)]


def grasp_scene(seed=0, n_fingers=4, links_per_finger=4, link_len=0.04, link_mass=0.05,
                link_radius=0.01, sphere_radius=0.05, sphere_cell=None, E=5e4, nu=0.45,
                rho=1000.0, mu=0.8, kp=5.0, kd=0.05, max_contacts=1024):
    """Articulated hand on a 6-DoF arm (3 prismatic + 3 revolute links of 1 kg, held by
    stiff drives) with four 4-link capsule fingers hanging around a tet-FEM sphere that
    rests on the ground.  Finger joints are PD-driven towards seeded sinusoids
    A sin(2 pi f t) (starting at the initial angle) that curl the fingers inwards onto
    the sphere and back."""
    rng = np.random.default_rng(seed)
    if sphere_cell is None:
        sphere_cell = 0.0108
    cz = sphere_radius + 1e-3
    sx, tets = sphere_tets(sphere_radius, sphere_cell, (0.0, 0.0, cz))
    sx[:, 2] += 1e-3 - sx[:, 2].min()  # voxelised sphere resting 1 mm above the ground
    d = _empty(mu=mu, max_contacts=max_contacts, name=f"grasp(seed={seed})")
    _set_tets(d, sx, tets, E, nu, rho)
    bodies, joints = [], []
    ex, ey, ez = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)
    finger_len = links_per_finger * link_len
    palm_half = (0.09, 0.09, 0.01)
    palm_bottom = finger_len + 2.0 * link_radius + 0.005
    palm_z = palm_bottom + palm_half[2]
    arm_z = palm_z + 0.1
    arm_h = (0.02, 0.02, 0.02)
    # arm: prismatic x, y, z from the world, then revolute z, y, x; stiff drives hold it
    prev = -1
    for a, axis in enumerate([ex, ey, ez]):
        bodies.append(_nocollide(_box(1.0, arm_h, (0.0, 0.0, arm_z))))
        idx = len(bodies) - 1
        anchor_prev = (0.0, 0.0, arm_z) if prev < 0 else (0.0, 0.0, 0.0)
        ref = [ey, ez, ex][a]
        joints.append(_prismatic(prev, idx, anchor_prev, (0.0, 0.0, 0.0), axis, axis, ref, ref,
                                 drive=(2e4, 2e2, rng.uniform(0.0, 0.01), rng.uniform(0.2, 1.0), 0.0, 0.0)))
        prev = idx
    for a, axis in enumerate([ez, ey, ex]):
        bodies.append(_nocollide(_box(1.0, arm_h, (0.0, 0.0, arm_z))))
        idx = len(bodies) - 1
        ref = ex if axis != ex else ey
        joints.append(_revolute(prev, idx, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), axis, axis, ref, ref,
                                drive=(500.0, 5.0, rng.uniform(0.0, 0.05), rng.uniform(0.2, 1.0), 0.0, 0.0)))
        prev = idx
    bodies.append(_box(0.2, palm_half, (0.0, 0.0, palm_z)))
    palm = len(bodies) - 1
    joints.append(_revolute(prev, palm, (0.0, 0.0, palm_z - arm_z), (0.0, 0.0, 0.0), ez, ez, ex, ex,
                            drive=(500.0, 5.0, 0.0, 0.5, 0.0, 0.0)))
    # fingers around the sphere; capsule axis = body x pointing down
    down = quat_from_axis_angle((0, 1, 0), math.pi / 2)
    R = _quat_to_mat(down)
    ring = sphere_radius + link_radius + 0.01
    corners = [(ring, 0.0), (-ring, 0.0), (0.0, ring), (0.0, -ring)][:n_fingers]
    for (fx, fy) in corners:
        inward = np.array([-fx, -fy, 0.0]) / ring
        hinge = np.cross(np.array([0.0, 0.0, -1.0]), inward)  # world; +angle curls inwards
        axis_link = tuple(R.T @ hinge)
        ref_link = tuple(R.T @ inward)
        parent = palm
        for l in range(links_per_finger):
            zc = palm_bottom - (l + 0.5) * link_len
            bodies.append(_capsule(link_mass, link_radius, 0.5 * link_len - link_radius,
                                   (fx, fy, zc), q=down))
            idx = len(bodies) - 1
            if parent == palm:
                anchor_parent, axis_parent, ref_parent = (fx, fy, -palm_half[2]), tuple(hinge), tuple(inward)
            else:
                anchor_parent, axis_parent, ref_parent = (0.5 * link_len, 0.0, 0.0), axis_link, ref_link
            joints.append(_revolute(parent, idx, anchor_parent, (-0.5 * link_len, 0.0, 0.0),
                                    axis_parent, axis_link, ref_parent, ref_link,
                                    drive=(kp, kd, rng.uniform(0.0, 0.6), rng.uniform(0.2, 1.0), 0.0, 0.0)))
            parent = idx
    _set_rigid(d, bodies)
    _set_joints(d, joints)
    return d.finalize()


def _quat_to_mat(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


# ----------------------------------------------------------------------------
# tiny cases with closed forms (used by the oracle's pins)
# ----------------------------------------------------------------------------

def free_particle(x=(0.0, 0.0, 1.0), v=(0.3, -0.2, 0.5), mass=2.0, gravity=(0.0, 0.0, -9.81)):
    d = _empty(n_particles=1, ground=0, gravity=gravity, name="free_particle")
    d.particle_x = np.array([x], np.float64)
    d.particle_rest = d.particle_x.copy()
    d.particle_v = np.array([v], np.float64)
    d.particle_mass = np.array([mass], np.float64)
    return d.finalize()


def particle_on_plane(v=(0.0, 0.0, 0.0), mass=1.0, mu=0.5, z=0.0, gravity=(0.0, 0.0, -9.81)):
    d = _empty(n_particles=1, mu=mu, gravity=gravity, name="particle_on_plane")
    d.particle_x = np.array([[0.1, -0.2, z]], np.float64)
    d.particle_rest = d.particle_x.copy()
    d.particle_v = np.array([v], np.float64)
    d.particle_mass = np.array([mass], np.float64)
    return d.finalize()


def spinning_box(w=(0.3, 2.0, -0.7), half=(0.1, 0.05, 0.2), mass=3.0):
    d = _empty(ground=0, gravity=(0.0, 0.0, 0.0), name="spinning_box")
    _set_rigid(d, [_box(mass, half, (0.0, 0.0, 1.0),
                        q=quat_from_axis_angle((1, 2, 3), 0.4), w=w, v=(0.1, 0.0, 0.0))])
    return d.finalize()


def box_on_incline(theta, mu, side=0.1, mass=1.0):
    """Dynamic cube resting on a static, tilted slab (the incline)."""
    slab_half = (1.0, 1.0, 0.05)
    q = quat_from_axis_angle((0, 1, 0), theta)
    R = _quat_to_mat(q)
    up = R @ np.array([0.0, 0.0, 1.0])
    slab_c = np.array([0.0, 0.0, 0.0])
    h = 0.5 * side
    box_c = slab_c + up * (slab_half[2] + h)
    d = _empty(mu=mu, ground=0, name=f"box_on_incline({theta:.3f},{mu})")
    _set_rigid(d, [_box(0.0, slab_half, slab_c, q=q), _box(mass, (h, h, h), box_c, q=q)])
    return d.finalize()


def particles_vs_planes_lcp(seed=0, n_particles=4, h=1.0 / 60.0):
    """Frictionless particles, each sitting in a corner of tilted static slabs so
    that up to three contacts share its three DOFs."""
    rng = np.random.default_rng(seed)
    bodies, px, pv = [], [], []
    for p in range(n_particles):
        base = np.array([3.0 * p, 0.0, 1.0])
        n_planes = 1 + p % 3
        for k in range(n_planes):
            nrm = rng.normal(size=3)
            nrm[2] = abs(nrm[2]) + 1.0
            nrm /= np.linalg.norm(nrm)
            # slab whose +z face passes through `base` with outward normal `nrm`
            ax = np.cross([0.0, 0.0, 1.0], nrm)
            ang = math.acos(np.clip(nrm[2], -1.0, 1.0))
            q = quat_from_axis_angle(ax, ang) if np.linalg.norm(ax) > 1e-9 else np.array([1.0, 0, 0, 0])
            bodies.append(_box(0.0, (0.5, 0.5, 0.05), base - nrm * 0.05, q=q))
        px.append(base + rng.normal(scale=1e-3, size=3) + np.array([0, 0, 1e-3]))
        pv.append(rng.normal(scale=0.3, size=3))
    d = _empty(mu=0.0, ground=0, name=f"particles_vs_planes(seed={seed})")
    _set_rigid(d, bodies)
    d.particle_x = np.array(px)
    d.particle_rest = d.particle_x.copy()
    d.particle_v = np.array(pv)
    d.particle_mass = rng.uniform(0.5, 2.0, size=n_particles)
    return d.finalize()


def single_tet(perturb=0.0, seed=0, E=1e5, nu=0.45, rho=1000.0, n_tets=1, gravity=(0.0, 0.0, 0.0),
               deform=None, tet_model=TET_NEOHOOKEAN):
    """1..5 tets from one hex (contact-free), optionally deformed by a matrix `deform`
    about the centroid and perturbed by noise of scale `perturb`."""
    rng = np.random.default_rng(seed)
    x, tets = hex_grid_tets(1, 1, 1, 0.1, origin=(0.0, 0.0, 1.0))
    tets = tets[:n_tets]
    used = np.unique(tets)
    remap = -np.ones(len(x), np.int64)
    remap[used] = np.arange(len(used))
    x = x[used]
    tets = remap[tets].astype(np.int32)
    d = _empty(ground=0, gravity=gravity, tet_model=tet_model, name=f"single_tet(n={n_tets})")
    _set_tets(d, x, tets, E, nu, rho)
    xd = x.copy()
    if deform is not None:
        c = x.mean(axis=0)
        xd = c + (x - c) @ np.asarray(deform, np.float64).T
    d.particle_x = xd + rng.normal(scale=perturb, size=x.shape)
    d.particle_v = rng.normal(scale=0.05, size=x.shape) if perturb > 0 else np.zeros_like(x)
    return d.finalize()


def pendulum_drive(kp=5.0, kd=0.05, amp=0.3, freq=0.5, phase=0.0, offset=0.0):
    """A box hinged to the world about the y axis at its centre, gravity-free, driven
    by an implicit PD drive towards a sinusoidal angle target."""
    d = _empty(ground=0, gravity=(0.0, 0.0, 0.0), name="pendulum_drive")
    _set_rigid(d, [_box(1.0, (0.1, 0.05, 0.05), (0.0, 0.0, 1.0))])
    _set_joints(d, [_revolute(-1, 0, (0.0, 0.0, 1.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 1.0, 0.0),
                              (1.0, 0.0, 0.0), (1.0, 0.0, 0.0), drive=(kp, kd, amp, freq, phase, offset))])
    return d.finalize()
