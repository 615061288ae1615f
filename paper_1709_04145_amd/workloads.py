"""Seeded synthetic workloads: articulated models and initial states.

This module only *describes inputs*.  It builds link trees, joint axes, joint
offsets and the per-link mass moment tensors of uniform boxes, and draws the
initial joint angles, torques and targets.  It holds none of the method's
arithmetic (no kinematics, objective, gradient or optimizer), so both the
FP64 CPU oracle and the HIP path consume exactly the same arrays from here.

Model description (all arrays are numpy, flat, C-contiguous):

* ``link_offset``  int32 [n_models+1]  links of model i are
  ``link_offset[i] .. link_offset[i+1]-1`` in the global link numbering.
* ``parent``       int32 [n_links]  parent link *within the model*
  (-1 = attached to the fixed world frame); parents precede children.
* ``dofs_per_link`` int32 [n_links]  1 (hinge) or 3 (ball joint = three
  consecutive hinges about the link-frame x, y, z axes).
* ``axis``         float64 [n_dofs, 3]  hinge axis of every DOF in the frame it
  rotates (unit vectors).  DOFs are numbered link-major.
* ``offset``       float64 [n_links, 3]  joint origin in the parent link frame
  (world frame for a root link).
* ``mass_moment``  float64 [n_links, 10]  upper triangle, row-major, of the
  symmetric 4x4 tensor  M = integral of rho (p;1)(p;1)^T dp  over the body:
  (M00 M01 M02 M03 M11 M12 M13 M22 M23 M33); units kg m^2, kg m, kg.
* ``gravity``      float64 [3]

Optional terms (None = absent; the applications of Sec. 6):

* ``dof_kind``     int32 [n_dofs]  0 = hinge (rotation about the axis), 1 = slide
  (translation along it).  A 6-DOF floating root is one link with three slides
  and three hinges (``dofs_per_link`` up to 6).
* ``drag``         float64 [n_links]  drag coefficient c_l >= 0 of the paper's drag
  potential (its D over the link's density).
* ``contact_link`` int32 [n_contacts] (global link index) and ``contact_point``
  float64 [n_contacts, 3] (link frame): discrete contact points of the penalty
  contact of Eq. FRI against the half-space n.x < h, ``contact_plane`` = (n, h),
  with penalties ``contact_d1`` (normal) and ``contact_d2`` (friction).

Every random draw uses ``numpy.random.default_rng([seed, i])`` per model i, so
the first n models of a configuration are identical whatever the batch size.
Model seeds are 1000+c and state seeds 2000+c for configuration c.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GRAVITY = np.array([0.0, 0.0, -9.81])


@dataclass
class ModelDesc:
    link_offset: np.ndarray
    parent: np.ndarray
    dofs_per_link: np.ndarray
    axis: np.ndarray
    offset: np.ndarray
    mass_moment: np.ndarray
    gravity: np.ndarray = field(default_factory=lambda: GRAVITY.copy())
    dof_kind: Optional[np.ndarray] = None
    drag: Optional[np.ndarray] = None
    contact_link: Optional[np.ndarray] = None
    contact_point: Optional[np.ndarray] = None
    contact_plane: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, 1.0, 0.0]))
    contact_d1: float = 0.0
    contact_d2: float = 0.0

    @property
    def n_contacts(self) -> int:
        return 0 if self.contact_link is None else int(self.contact_link.shape[0])

    @property
    def has_extras(self) -> bool:
        """Slides, drag or contact points present."""
        return (self.dof_kind is not None and bool(np.any(self.dof_kind != 0))) or \
            (self.drag is not None and bool(np.any(self.drag != 0))) or self.n_contacts > 0

    @property
    def n_models(self) -> int:
        return int(self.link_offset.shape[0] - 1)

    @property
    def n_links(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_dofs(self) -> int:
        return int(self.axis.shape[0])

    @property
    def dof_offset(self) -> np.ndarray:
        """int32 [n_models+1]: DOFs of model i are dof_offset[i]..dof_offset[i+1]-1."""
        per_link = np.concatenate([[0], np.cumsum(self.dofs_per_link)]).astype(np.int64)
        return per_link[self.link_offset].astype(np.int32)

    @property
    def link_dof_start(self) -> np.ndarray:
        """int32 [n_links]: global index of the first DOF of every link."""
        return np.concatenate([[0], np.cumsum(self.dofs_per_link)[:-1]]).astype(np.int32)

    def links_of(self, i: int) -> int:
        return int(self.link_offset[i + 1] - self.link_offset[i])

    def subset(self, models) -> "ModelDesc":
        """A new description holding only the listed models (in that order)."""
        models = np.asarray(models, dtype=np.int64)
        lo, do = self.link_offset, self.dof_offset
        link_idx = np.concatenate([np.arange(lo[m], lo[m + 1]) for m in models])
        dof_idx = np.concatenate([np.arange(do[m], do[m + 1]) for m in models])
        counts = np.array([lo[m + 1] - lo[m] for m in models])
        out = ModelDesc(
            link_offset=np.concatenate([[0], np.cumsum(counts)]).astype(np.int32),
            parent=self.parent[link_idx].copy(),
            dofs_per_link=self.dofs_per_link[link_idx].copy(),
            axis=self.axis[dof_idx].copy(),
            offset=self.offset[link_idx].copy(),
            mass_moment=self.mass_moment[link_idx].copy(),
            gravity=self.gravity.copy(),
            dof_kind=None if self.dof_kind is None else self.dof_kind[dof_idx].copy(),
            drag=None if self.drag is None else self.drag[link_idx].copy(),
            contact_plane=self.contact_plane.copy(), contact_d1=self.contact_d1, contact_d2=self.contact_d2,
        )
        if self.n_contacts:
            new_of = np.full(self.n_links, -1, np.int64)
            new_of[link_idx] = np.arange(link_idx.shape[0])
            keep = new_of[self.contact_link] >= 0
            # contacts ordered as the models of the subset
            order = np.argsort(new_of[self.contact_link][keep], kind="stable")
            out.contact_link = new_of[self.contact_link][keep][order].astype(np.int32)
            out.contact_point = self.contact_point[keep][order].copy()
        return out

    def dof_subset_index(self, models) -> np.ndarray:
        do = self.dof_offset
        return np.concatenate([np.arange(do[m], do[m + 1]) for m in np.asarray(models)])


def box_mass_moment(length: float, width: float, density: float) -> np.ndarray:
    """Upper triangle of M for a box spanning x in [0,L], y,z in [-w/2,w/2]."""
    m = density * length * width * width
    return np.array([
        m * length * length / 3.0, 0.0, 0.0, m * length / 2.0,
        m * width * width / 12.0, 0.0, 0.0,
        m * width * width / 12.0, 0.0,
        m,
    ])


def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v)


def _assemble(models) -> ModelDesc:
    """models: list of dicts with parent, dofs, axis, offset, mm (per model)."""
    if not models:
        return ModelDesc(link_offset=np.zeros(1, np.int32), parent=np.zeros(0, np.int32),
                         dofs_per_link=np.zeros(0, np.int32), axis=np.zeros((0, 3)),
                         offset=np.zeros((0, 3)), mass_moment=np.zeros((0, 10)),
                         gravity=GRAVITY.copy())
    counts = [len(m["parent"]) for m in models]
    return ModelDesc(
        link_offset=np.concatenate([[0], np.cumsum(counts)]).astype(np.int32),
        parent=np.concatenate([m["parent"] for m in models]).astype(np.int32),
        dofs_per_link=np.concatenate([m["dofs"] for m in models]).astype(np.int32),
        axis=np.ascontiguousarray(np.concatenate([m["axis"] for m in models]), dtype=np.float64),
        offset=np.ascontiguousarray(np.concatenate([m["offset"] for m in models]), dtype=np.float64),
        mass_moment=np.ascontiguousarray(np.concatenate([m["mm"] for m in models]), dtype=np.float64),
        gravity=GRAVITY.copy(),
    )


def chain_model(lengths, width, densities, axes) -> dict:
    """One serial chain: root joint at the world origin, child joint at (L,0,0)."""
    n = len(lengths)
    offset = np.zeros((n, 3))
    for l in range(1, n):
        offset[l, 0] = lengths[l - 1]
    return dict(
        parent=np.arange(-1, n - 1),
        dofs=np.ones(n, dtype=np.int32),
        axis=np.asarray(axes, dtype=np.float64).reshape(n, 3),
        offset=offset,
        mm=np.stack([box_mass_moment(lengths[l], width, densities[l]) for l in range(n)]),
    )


def alternating_axes(n: int, first: str = "x") -> np.ndarray:
    ex, ey = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    a, b = (ex, ey) if first == "x" else (ey, ex)
    return np.stack([a if l % 2 == 0 else b for l in range(n)])


def tree_model(parent, length, width, density) -> dict:
    """Tree of ball-jointed links; each child attaches at its parent's (L,0,0)."""
    n = len(parent)
    offset = np.zeros((n, 3))
    for l in range(n):
        if parent[l] >= 0:
            offset[l, 0] = length
    axis = np.tile(np.eye(3), (n, 1))
    return dict(
        parent=np.asarray(parent),
        dofs=np.full(n, 3, dtype=np.int32),
        axis=axis,
        offset=offset,
        mm=np.tile(box_mass_moment(length, width, density), (n, 1)),
    )


def bfs_tree_parents(n: int, rng: np.random.Generator) -> np.ndarray:
    """Breadth-first random tree: pop a node, give it min(c, remaining) children, c~U{1..3}."""
    parent = [-1]
    queue = [0]
    head = 0
    while len(parent) < n:
        node = queue[head]
        head += 1
        c = int(rng.integers(1, 4))
        for _ in range(min(c, n - len(parent))):
            parent.append(node)
            queue.append(len(parent) - 1)
    return np.array(parent, dtype=np.int32)


@dataclass
class StepConfig:
    dt: float
    steps: int
    order_K: int = 2
    lbfgs_m: int = 5
    tol: float = 1e-8
    max_iter: int = 500


@dataclass
class Workload:
    name: str
    model: ModelDesc
    q0: np.ndarray                      # [n_dofs] initial angles (zero velocity)
    step: StepConfig
    torque: Optional[np.ndarray] = None  # [steps, n_dofs] (config 5)
    target: Optional[np.ndarray] = None  # [n_models, 3] (config 5)


CONFIG_NAMES = {
    1: "chain10_fp64",
    2: "chains4096_uneven10to50",
    3: "trees2048_ball_K4",
    4: "ropes256x1000",
    5: "chains4096_torque_grad",
    6: "swimmers8192_drag",
    7: "spiders4096_contact",
}


def config_models(c: int, n_models: Optional[int] = None) -> ModelDesc:
    seed = 1000 + c
    models = []
    if c == 1:
        n = 10
        models.append(chain_model([1.0] * n, 0.1, [1000.0] * n, alternating_axes(n)))
    elif c in (2, 5):
        total = 4096 if n_models is None else n_models
        for i in range(total):
            rng = np.random.default_rng([seed, i])
            n = int(rng.integers(10, 51))
            if c == 2:
                lengths = rng.uniform(0.3, 1.2, n)
                dens = rng.uniform(500.0, 2000.0, n)
                axes = np.stack([_unit(rng.standard_normal(3)) for _ in range(n)])
                models.append(chain_model(lengths, 0.1, dens, axes))
            else:
                models.append(chain_model([1.0] * n, 0.1, [1000.0] * n, alternating_axes(n)))
    elif c == 3:
        total = 2048 if n_models is None else n_models
        for i in range(total):
            rng = np.random.default_rng([seed, i])
            n = int(rng.integers(30, 61))
            models.append(tree_model(bfs_tree_parents(n, rng), 1.0, 0.1, 1000.0))
    elif c == 4:
        total = 256 if n_models is None else n_models
        for i in range(total):
            n = 1000
            models.append(chain_model([0.05] * n, 0.01, [1000.0] * n, alternating_axes(n)))
    elif c == 6:
        return swimmer_models(8192 if n_models is None else n_models, seed)
    elif c == 7:
        return spider_models(4096 if n_models is None else n_models, seed)
    else:
        raise ValueError(f"unknown configuration {c}")
    if c == 1 and n_models not in (None, 1):
        raise ValueError("configuration 1 has a single model")
    return _assemble(models)


_Q_RANGE = {1: 0.5, 2: 1.0, 3: 0.5, 4: 0.2, 5: 0.5, 6: 0.5, 7: 0.05}
_STEP = {
    1: StepConfig(dt=0.01, steps=100, order_K=2, lbfgs_m=5, tol=1e-8),
    2: StepConfig(dt=0.03, steps=100, order_K=2, lbfgs_m=5, tol=1e-8),
    3: StepConfig(dt=0.05, steps=50, order_K=4, lbfgs_m=5, tol=1e-8),
    4: StepConfig(dt=0.1, steps=200, order_K=2, lbfgs_m=10, tol=1e-8),
    5: StepConfig(dt=0.03, steps=50, order_K=2, lbfgs_m=5, tol=1e-8),
    6: StepConfig(dt=0.05, steps=100, order_K=2, lbfgs_m=5, tol=1e-8),
    # contact steps: the float64 floor of the resting spiders' gradient lies near
    # 1e-8 of its warm-start value, so the tolerance is 1e-6 (every step converges
    # within 200 iterations in the oracle)
    7: StepConfig(dt=0.01, steps=100, order_K=2, lbfgs_m=5, tol=1e-6, max_iter=1000),
}
# configuration 6: joint torques on the swimmers' three body hinges, U(-0.2, 0.2) N m
SWIM_TORQUE = 0.2
# configuration 7: torso height of the standing pose (every foot 1..5 cm above the ground)
SPIDER_HEIGHT = 0.34


def config(c: int, n_models: Optional[int] = None, steps: Optional[int] = None) -> Workload:
    """Configuration c (1..7); n_models truncates the batch to its first models."""
    model = config_models(c, n_models)
    sc = StepConfig(**vars(_STEP[c]))
    if steps is not None:
        sc.steps = steps
    a = _Q_RANGE[c]
    seed = 2000 + c
    dof_off = model.dof_offset
    q0 = np.empty(model.n_dofs)
    torque = np.empty((sc.steps, model.n_dofs)) if c in (5, 6) else None
    target = np.empty((model.n_models, 3)) if c == 5 else None
    for i in range(model.n_models):
        rng = np.random.default_rng([seed, i])
        d0, d1 = dof_off[i], dof_off[i + 1]
        q0[d0:d1] = rng.uniform(-a, a, d1 - d0)
        if c == 6:
            # root near the origin, body hinges within +-a; torques on the body hinges only
            q0[d0:d0 + 3] = rng.uniform(-0.1, 0.1, 3)
            q0[d0 + 3:d0 + 6] = rng.uniform(-0.2, 0.2, 3)
            torque[:, d0:d1] = 0.0
            torque[:, d0 + 6:d1] = (SWIM_TORQUE * rng.uniform(-1.0, 1.0, (sc.steps, 3))).astype(np.float32)
        if c == 7:
            # standing pose: torso level at SPIDER_HEIGHT; legs out at +-45 / +-135
            # degrees, thighs pitched down, knees bent by 1 rad, each angle within +-a
            q0[d0:d0 + 6] = [0.0, 0.0, SPIDER_HEIGHT, 0.0, 0.0, 0.0]
            for leg, phi in enumerate((np.pi / 4, -np.pi / 4, 3 * np.pi / 4, -3 * np.pi / 4)):
                b = d0 + 6 + 4 * leg
                q0[b + 1] += 0.5 * np.sign(np.cos(phi))
                q0[b + 2] += phi
                q0[b + 3] += 1.0
        if c == 5:
            # FP32 torques, stored exactly in float64
            torque[:, d0:d1] = rng.uniform(-1.0, 1.0, (sc.steps, d1 - d0)).astype(np.float32)
            direction = _unit(rng.standard_normal(3))
            target[i] = direction * 2.0 * rng.uniform() ** (1.0 / 3.0)
    return Workload(CONFIG_NAMES[c], model, q0, sc, torque, target)


def random_tree_models(n_models: int, seed: int, max_links: int = 6, ball_prob: float = 0.3,
                       gravity=None) -> ModelDesc:
    """Small random trees with mixed hinge / ball joints and random geometry (tests)."""
    models = []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(1, max_links + 1))
        parent = np.array([-1] + [int(rng.integers(0, l)) for l in range(1, n)])
        dofs = np.where(rng.uniform(size=n) < ball_prob, 3, 1).astype(np.int32)
        axis = []
        for l in range(n):
            if dofs[l] == 3:
                axis.extend(list(np.eye(3)))
            else:
                axis.append(_unit(rng.standard_normal(3)))
        lengths = rng.uniform(0.2, 1.0, n)
        offset = np.zeros((n, 3))
        offset[0] = rng.uniform(-0.5, 0.5, 3)
        for l in range(1, n):
            offset[l] = [lengths[parent[l]], *rng.uniform(-0.05, 0.05, 2)]
        mm = np.stack([box_mass_moment(lengths[l], rng.uniform(0.05, 0.2),
                                       rng.uniform(500, 2000)) for l in range(n)])
        models.append(dict(parent=parent, dofs=dofs, axis=np.array(axis), offset=offset, mm=mm))
    desc = _assemble(models)
    if gravity is not None:
        desc.gravity = np.asarray(gravity, dtype=np.float64)
    return desc


def _with_extras(models, kinds=None, drag=None, contacts=None, gravity=None, plane=None, d1=0.0, d2=0.0):
    """_assemble plus the optional terms: kinds / drag per model (lists of arrays),
    contacts per model as (local link index, point) lists."""
    desc = _assemble(models)
    if kinds is not None:
        desc.dof_kind = np.concatenate(kinds).astype(np.int32)
    if drag is not None:
        desc.drag = np.concatenate(drag).astype(np.float64)
    if contacts is not None:
        links, pts = [], []
        for i, cs in enumerate(contacts):
            for l, p in cs:
                links.append(int(desc.link_offset[i]) + l)
                pts.append(p)
        if links:
            desc.contact_link = np.array(links, dtype=np.int32)
            desc.contact_point = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    if gravity is not None:
        desc.gravity = np.asarray(gravity, dtype=np.float64)
    if plane is not None:
        desc.contact_plane = np.asarray(plane, dtype=np.float64)
    desc.contact_d1, desc.contact_d2 = float(d1), float(d2)
    return desc


# a 6-DOF floating root: slides along the parent (world) x, y, z, then hinges about x, y, z
FREE_KINDS = np.array([1, 1, 1, 0, 0, 0], dtype=np.int32)
FREE_AXES = np.concatenate([np.eye(3), np.eye(3)])


def swimmer_models(n_models: int, seed: int, drag=(0.02, 0.1)) -> ModelDesc:
    """Swimmers of the paper's controller benchmark (Sec. 6): a chain of four links
    (boxes 0.3..0.4 m long, 5 cm wide, density 1000) on a 6-DOF floating root,
    three hinges about the link z axes (9 DOFs), the drag potential on every
    link with c ~ U[drag], no gravity (neutrally buoyant)."""
    models, kinds, drags = [], [], []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        lengths = rng.uniform(0.3, 0.4, 4)
        offset = np.zeros((4, 3))
        offset[1:, 0] = lengths[:3]
        models.append(dict(parent=np.arange(-1, 3), dofs=np.array([6, 1, 1, 1], np.int32),
                           axis=np.concatenate([FREE_AXES, np.tile([0.0, 0.0, 1.0], (3, 1))]),
                           offset=offset,
                           mm=np.stack([box_mass_moment(L, 0.05, 1000.0) for L in lengths])))
        kinds.append(np.concatenate([FREE_KINDS, np.zeros(3, np.int32)]))
        drags.append(np.full(4, rng.uniform(*drag)))
    return _with_extras(models, kinds=kinds, drag=drags, gravity=[0.0, 0.0, 0.0])


SPIDER_D1, SPIDER_D2 = 2.0e4, 2.0e5


def spider_models(n_models: int, seed: int) -> ModelDesc:
    """Spiders of the paper's controller benchmark (Sec. 6): a torso (box 0.3 x
    0.15 x 0.15 m, density 300) on a 6-DOF floating root and four legs, each a
    thigh (0.18..0.22 m) on a ball hip at a torso corner and a shin
    (0.22..0.28 m) on a knee hinge about the thigh's y axis (22 DOFs: the
    paper's joint list), under gravity, with the penalty contact of Eq. FRI at
    the four feet and the torso's four lower corners against the ground z < 0."""
    models, kinds, contacts = [], [], []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        L, w = 0.3, 0.15
        thigh = rng.uniform(0.18, 0.22, 4)
        shin = rng.uniform(0.22, 0.28, 4)
        parent, dofs, axis, offset, mm, cs = [-1], [6], [FREE_AXES], [np.zeros(3)], \
            [box_mass_moment(L, w, 300.0)], []
        corners = [(0.25, 0.075), (0.25, -0.075), (0.05, 0.075), (0.05, -0.075)]
        for leg, (cx, cy) in enumerate(corners):
            parent.append(0)
            dofs.append(3)
            axis.append(np.eye(3))
            offset.append(np.array([cx, cy, 0.0]))
            mm.append(box_mass_moment(thigh[leg], 0.03, 1000.0))
            parent.append(len(parent) - 1)
            dofs.append(1)
            axis.append(np.array([[0.0, 1.0, 0.0]]))
            offset.append(np.array([thigh[leg], 0.0, 0.0]))
            mm.append(box_mass_moment(shin[leg], 0.02, 1000.0))
            cs.append((len(parent) - 1, [shin[leg], 0.0, 0.0]))
        for x in (0.0, L):
            for y in (-w / 2, w / 2):
                cs.append((0, [x, y, -w / 2]))
        models.append(dict(parent=np.array(parent), dofs=np.array(dofs, np.int32), axis=np.concatenate(axis),
                           offset=np.stack(offset), mm=np.stack(mm)))
        kinds.append(np.concatenate([FREE_KINDS, np.zeros(16, np.int32)]))
        contacts.append(cs)
    return _with_extras(models, kinds=kinds, contacts=contacts, plane=[0.0, 0.0, 1.0, 0.0],
                        d1=SPIDER_D1, d2=SPIDER_D2)


def random_extras_models(n_models: int, seed: int, max_links: int = 5, d1: float = 2.0e3,
                         d2: float = 1.0e4) -> ModelDesc:
    """Small random trees (tests) whose links mix hinges, ball joints, slides and
    floating roots, with random drag on some links and contact points on some
    links against the plane z < -0.2."""
    models, kinds, drags, contacts = [], [], [], []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(1, max_links + 1))
        parent = np.array([-1] + [int(rng.integers(0, l)) for l in range(1, n)])
        dofs, axis, kind = [], [], []
        for l in range(n):
            u = rng.uniform()
            if l == 0 and u < 0.5:
                dofs.append(6)
                axis.append(FREE_AXES)
                kind.append(FREE_KINDS)
            elif u < 0.25:
                dofs.append(1)
                axis.append(_unit(rng.standard_normal(3))[None, :])
                kind.append(np.ones(1, np.int32))
            elif u < 0.5:
                dofs.append(3)
                axis.append(np.eye(3))
                kind.append(np.zeros(3, np.int32))
            else:
                dofs.append(1)
                axis.append(_unit(rng.standard_normal(3))[None, :])
                kind.append(np.zeros(1, np.int32))
        lengths = rng.uniform(0.2, 1.0, n)
        offset = np.zeros((n, 3))
        offset[0] = rng.uniform(-0.3, 0.3, 3)
        for l in range(1, n):
            offset[l] = [lengths[parent[l]], *rng.uniform(-0.05, 0.05, 2)]
        mm = np.stack([box_mass_moment(lengths[l], rng.uniform(0.05, 0.2), rng.uniform(500, 2000))
                       for l in range(n)])
        models.append(dict(parent=parent, dofs=np.array(dofs, np.int32), axis=np.concatenate(axis),
                           offset=offset, mm=mm))
        kinds.append(np.concatenate(kind))
        drags.append(np.where(rng.uniform(size=n) < 0.5, rng.uniform(0.0, 0.3, n), 0.0))
        contacts.append([(l, [lengths[l] * rng.uniform(), *rng.uniform(-0.05, 0.05, 2)])
                         for l in range(n) for _ in range(int(rng.integers(0, 3)))])
    return _with_extras(models, kinds=kinds, drag=drags, contacts=contacts, plane=[0.0, 0.0, 1.0, -0.2],
                        d1=d1, d2=d2)


def random_chain_models(n_models: int, seed: int, lo: int = 1, hi: int = 64) -> ModelDesc:
    """Random hinge chains with link counts in [lo, hi] (tests: ragged batches)."""
    models = []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(lo, hi + 1))
        lengths = rng.uniform(0.3, 1.2, n)
        dens = rng.uniform(500.0, 2000.0, n)
        axes = np.stack([_unit(rng.standard_normal(3)) for _ in range(n)])
        models.append(chain_model(lengths, 0.1, dens, axes))
    return _assemble(models)


def random_state(model: ModelDesc, seed: int, spread: float = 1.0, velocity: float = 0.0):
    """(q_prev, q_curr) with q_curr ~ U[-spread, spread], q_prev = q_curr - velocity*noise."""
    rng = np.random.default_rng(seed)
    q1 = rng.uniform(-spread, spread, model.n_dofs)
    q0 = q1 - velocity * rng.uniform(-1.0, 1.0, model.n_dofs)
    return q0, q1
