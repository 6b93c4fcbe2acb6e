"""Seeded synthetic mesh generators for the cell-centred FVLBM.

These build the raw unstructured meshes that both the HIP library and the
FP64 oracle take as input: node coordinates, CCW cell->node lists, boundary
edges with their boundary-condition group, and periodic edge pairs.  The
module holds no arithmetic of the method itself (no areas, normals,
gradients or fluxes); it only places nodes and writes connectivity.

Mesh classes follow the paper's workloads (Section 3): plate-driven Couette
flow on a periodic channel, the lid-driven cavity on wall-clustered
triangles, body-fitted O-grids around one or two circular cylinders.  The
paper's own meshes were made with an external mesher and are not available,
so these are stand-ins of the same shape, size and structure.

Boundary-condition kinds (Section 2.4): WALL, INLET, OUTLET, SYMMETRY.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

WALL, INLET, OUTLET, SYMMETRY = 1, 2, 3, 4


@dataclasses.dataclass
class BCGroup:
    kind: int
    u: tuple = (0.0, 0.0)      # wall velocity u_w, or free-stream u_inf
    rho: float = 1.0           # rho_inf for inlet / outlet
    internal: int = 0          # 0: external flow, 1: internal flow (velocity inlet / pressure outlet)


@dataclasses.dataclass
class RawMesh:
    nodes: np.ndarray          # (n_nodes, 2) float64
    cell_ptr: np.ndarray       # (n_cells + 1,) int32, CSR
    cell_nodes: np.ndarray     # int32, CCW per cell
    bface_nodes: np.ndarray    # (n_bfaces, 2) int32, unordered node pair of a boundary edge
    bface_group: np.ndarray    # (n_bfaces,) int32, index into groups; -1 for periodic edges
    groups: List[BCGroup]
    periodic: np.ndarray       # (n_per, 2) int32: boundary-edge indices (a, b) joined by periodicity
    periodic_shift: np.ndarray  # (n_per, 2) float64: add to positions on b's side to bring them next to a
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.cell_ptr.shape[0] - 1)

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    def nodes_per_cell(self) -> np.ndarray:
        return np.diff(self.cell_ptr)


# --------------------------------------------------------------------------
# helpers (connectivity only)
# --------------------------------------------------------------------------

def _structured_nodes(xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # [j, i]
    return np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)


def _nid(i, j, nx1):
    return j * nx1 + i


def _signed_area2(p0, p1, p2):
    """Twice the signed area of a triangle; used only to reject inverted jitter draws."""
    return (p1[..., 0] - p0[..., 0]) * (p2[..., 1] - p0[..., 1]) - \
           (p2[..., 0] - p0[..., 0]) * (p1[..., 1] - p0[..., 1])


def _rect_cells(nx, ny, tri: bool, diag: str = "ll-ur"):
    """CCW quads or triangles of an (nx x ny) structured block; node (i,j) = j*(nx+1)+i."""
    nx1 = nx + 1
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ii = ii.ravel(); jj = jj.ravel()
    a = _nid(ii, jj, nx1); b = _nid(ii + 1, jj, nx1)
    c = _nid(ii + 1, jj + 1, nx1); d = _nid(ii, jj + 1, nx1)
    if not tri:
        cells = np.stack([a, b, c, d], axis=1)
        ptr = np.arange(0, 4 * cells.shape[0] + 1, 4, dtype=np.int32)
        return ptr, cells.ravel().astype(np.int32)
    # split each quad along its (i,j)-(i+1,j+1) diagonal: two CCW triangles
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    cells = np.stack([t1, t2], axis=1).reshape(-1, 3)
    ptr = np.arange(0, 3 * cells.shape[0] + 1, 3, dtype=np.int32)
    return ptr, cells.ravel().astype(np.int32)


def _rect_boundary(nx, ny, side_group, periodic_x=False, periodic_y=False,
                   Lx=1.0, Ly=1.0):
    """Boundary edges of a structured rectangle.

    side_group maps 'bottom','right','top','left' to a group index (ignored for
    periodic sides).  Returns (bface_nodes, bface_group, periodic, shift).
    """
    nx1 = nx + 1
    bf, grp = [], []
    side_ids = {}
    for s in ("bottom", "right", "top", "left"):
        ids = []
        if s == "bottom":
            for i in range(nx):
                ids.append(len(bf)); bf.append((_nid(i, 0, nx1), _nid(i + 1, 0, nx1)))
        elif s == "top":
            for i in range(nx):
                ids.append(len(bf)); bf.append((_nid(i, ny, nx1), _nid(i + 1, ny, nx1)))
        elif s == "left":
            for j in range(ny):
                ids.append(len(bf)); bf.append((_nid(0, j, nx1), _nid(0, j + 1, nx1)))
        else:
            for j in range(ny):
                ids.append(len(bf)); bf.append((_nid(nx, j, nx1), _nid(nx, j + 1, nx1)))
        periodic_side = (periodic_x and s in ("left", "right")) or (periodic_y and s in ("bottom", "top"))
        g = -1 if periodic_side else side_group[s]
        grp.extend([g] * len(ids))
        side_ids[s] = ids
    per, shift = [], []
    if periodic_x:
        for a, b in zip(side_ids["left"], side_ids["right"]):
            per.append((a, b)); shift.append((-Lx, 0.0))      # right-side cell seen from the left edge
    if periodic_y:
        for a, b in zip(side_ids["bottom"], side_ids["top"]):
            per.append((a, b)); shift.append((0.0, -Ly))
    return (np.asarray(bf, dtype=np.int32), np.asarray(grp, dtype=np.int32),
            np.asarray(per, dtype=np.int32).reshape(-1, 2),
            np.asarray(shift, dtype=np.float64).reshape(-1, 2))


def _tanh_points(n: int, beta: float) -> np.ndarray:
    s = 2.0 * np.arange(n + 1) / n - 1.0
    p = 0.5 * (1.0 + np.tanh(beta * s) / np.tanh(beta))
    p[0], p[-1] = 0.0, 1.0
    return p


def tanh_beta(n: int, ratio: float) -> float:
    """Stretching parameter beta of x = (1 + tanh(beta (2i/n - 1))/tanh beta)/2 giving a
    wall growth ratio h1/h0 = ratio on n cells."""
    def growth(beta):
        p = _tanh_points(n, beta)
        return (p[2] - p[1]) / (p[1] - p[0])
    lo, hi = 1e-6, 12.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if growth(mid) < ratio:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def tanh_cluster(n: int, ratio: float, beta: Optional[float] = None) -> np.ndarray:
    """n+1 points on [0,1], tanh-clustered at both ends: wall growth ratio h1/h0 = ratio,
    or the given stretching parameter beta."""
    if beta is None:
        if ratio <= 1.0:
            return np.linspace(0.0, 1.0, n + 1)
        beta = tanh_beta(n, ratio)
    return _tanh_points(n, beta)


def solve_geometric_ratio(h0: float, n: int, length: float) -> float:
    """Ratio q with h0 (q^n - 1)/(q - 1) = length."""
    def tot(q):
        return h0 * n if abs(q - 1.0) < 1e-14 else h0 * (q ** n - 1.0) / (q - 1.0)
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        if tot(mid) < length:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def couette(nx: int = 16, ny: int = 16, U: float = 0.1, tri: bool = False,
            Lx: float = 1.0, Ly: float = 1.0) -> RawMesh:
    """Plate-driven Couette channel (Section 3.1): periodic in x, bottom wall at rest,
    top wall moving at (U, 0)."""
    xs = np.linspace(0.0, Lx, nx + 1); ys = np.linspace(0.0, Ly, ny + 1)
    nodes = _structured_nodes(xs, ys)
    ptr, cells = _rect_cells(nx, ny, tri)
    groups = [BCGroup(WALL, (0.0, 0.0)), BCGroup(WALL, (U, 0.0))]
    bf, grp, per, sh = _rect_boundary(nx, ny, {"bottom": 0, "top": 1, "left": -1, "right": -1},
                                      periodic_x=True, Lx=Lx, Ly=Ly)
    return RawMesh(nodes, ptr, cells, bf, grp, groups, per, sh,
                   name=f"couette_{nx}x{ny}_{'tri' if tri else 'quad'}",
                   meta=dict(U=U, L=Ly, kind="couette"))


def cavity(n: int = 100, ratio: float = 1.08, jitter: float = 0.2, seed: int = 0,
           lid_u: float = 0.1, tri: bool = True, beta: Optional[float] = None) -> RawMesh:
    """Lid-driven square cavity (Section 3.2): tanh wall clustering with growth ratio
    `ratio` (or stretching parameter `beta`), quads split into triangles along the
    (i,j)-(i+1,j+1) diagonal, interior nodes jittered by +-`jitter` x local spacing
    from `seed`.  Top wall moves at lid_u."""
    xs = tanh_cluster(n, ratio, beta); ys = xs.copy()
    nodes = _structured_nodes(xs, ys)
    ptr, cells = _rect_cells(n, n, tri)
    rng = np.random.default_rng(seed)
    if jitter > 0.0:
        nodes = _jitter_fast(nodes, xs, ys, n, n, jitter, rng, tri)
    groups = [BCGroup(WALL, (0.0, 0.0)), BCGroup(WALL, (lid_u, 0.0))]
    bf, grp, per, sh = _rect_boundary(n, n, {"bottom": 0, "right": 0, "left": 0, "top": 1})
    return RawMesh(nodes, ptr, cells, bf, grp, groups, per, sh,
                   name=f"cavity_{n}_{'tri' if tri else 'quad'}_s{seed}",
                   meta=dict(U=lid_u, L=1.0, kind="cavity", seed=seed))


def _jitter_fast(nodes, xs, ys, nx, ny, amp, rng, tri):
    """Vectorised interior-node jitter for structured-topology meshes.

    Same rule as _jitter_interior (U(-amp,amp) x local spacing per direction;
    redraw any node whose incident cells would invert), checked on the
    structured stencil so it scales to millions of cells.
    """
    nx1 = nx + 1
    dx = np.diff(xs); dy = np.diff(ys)
    out = nodes.reshape(ny + 1, nx1, 2).copy()
    sx = np.minimum(dx[:-1], dx[1:])[None, :]          # interior i=1..nx-1
    sy = np.minimum(dy[:-1], dy[1:])[:, None]          # interior j=1..ny-1
    base = out[1:ny, 1:nx].copy()
    todo = np.ones(base.shape[:2], dtype=bool)
    for it in range(60):
        if not todo.any():
            break
        ox = rng.uniform(-amp, amp, size=todo.shape) * sx
        oy = rng.uniform(-amp, amp, size=todo.shape) * sy
        cand = out[1:ny, 1:nx].copy()
        cand[..., 0] = np.where(todo, base[..., 0] + ox, cand[..., 0])
        cand[..., 1] = np.where(todo, base[..., 1] + oy, cand[..., 1])
        trial = out.copy(); trial[1:ny, 1:nx] = cand
        bad = _bad_nodes(trial, nx, ny, tri)
        # accept the draws of nodes that touch no inverted cell; retry the others
        accept = todo & ~bad[1:ny, 1:nx]
        out[1:ny, 1:nx][accept] = cand[accept]
        todo &= ~accept
        if it == 59:
            out[1:ny, 1:nx][todo] = base[todo]
    # a node that touched a bad cell only through a neighbour still pending is
    # re-checked globally: revert any node still adjacent to an inverted cell
    for _ in range(10):
        bad = _bad_nodes(out, nx, ny, tri)
        if not bad.any():
            break
        mask = bad.copy(); mask[0, :] = mask[-1, :] = False; mask[:, 0] = mask[:, -1] = False
        orig = _structured_nodes(xs, ys).reshape(ny + 1, nx1, 2)
        out[mask] = orig[mask]
    return out.reshape(-1, 2)


def _bad_nodes(P, nx, ny, tri):
    """Boolean (ny+1, nx+1) mask of nodes incident to a cell with a non-positive corner."""
    a = P[:-1, :-1]; b = P[:-1, 1:]; c = P[1:, 1:]; d = P[1:, :-1]
    if tri:
        cells = [(a, b, c), (a, c, d)]
    else:
        cells = [(a, b, c, d)]
    bad_cell = np.zeros((ny, nx), dtype=bool)
    for cv in cells:
        m = len(cv)
        for k in range(m):
            bad_cell |= _signed_area2(cv[k - 1], cv[k], cv[(k + 1) % m]) <= 0.0
    bad = np.zeros((ny + 1, nx + 1), dtype=bool)
    bad[:-1, :-1] |= bad_cell; bad[:-1, 1:] |= bad_cell
    bad[1:, 1:] |= bad_cell; bad[1:, :-1] |= bad_cell
    return bad


def periodic_box(nx: int = 12, ny: int = 12, jitter: float = 0.2, seed: int = 0,
                 tri: bool = True, Lx: float = 1.0, Ly: float = 1.0) -> RawMesh:
    """Doubly periodic box; interior nodes jittered, boundary nodes fixed so the
    periodic edge pairs stay congruent."""
    xs = np.linspace(0.0, Lx, nx + 1); ys = np.linspace(0.0, Ly, ny + 1)
    nodes = _structured_nodes(xs, ys)
    ptr, cells = _rect_cells(nx, ny, tri)
    if jitter > 0.0:
        nodes = _jitter_fast(nodes, xs, ys, nx, ny, jitter, np.random.default_rng(seed), tri)
    bf, grp, per, sh = _rect_boundary(nx, ny, {}, periodic_x=True, periodic_y=True, Lx=Lx, Ly=Ly)
    return RawMesh(nodes, ptr, cells, bf, grp, [], per, sh,
                   name=f"pbox_{nx}x{ny}_{'tri' if tri else 'quad'}_s{seed}",
                   meta=dict(kind="pbox", seed=seed))


def channel(nx: int = 24, ny: int = 12, u_in=(0.1, 0.0), rho_inf: float = 1.0,
            internal: int = 0, top: str = "wall", bottom: str = "wall",
            jitter: float = 0.0, seed: int = 0, tri: bool = False,
            Lx: float = 2.0, Ly: float = 1.0) -> RawMesh:
    """Rectangular channel: inlet on the left, outlet on the right, top/bottom
    walls at rest (or symmetry planes, or far-field inlets)."""
    xs = np.linspace(0.0, Lx, nx + 1); ys = np.linspace(0.0, Ly, ny + 1)
    nodes = _structured_nodes(xs, ys)
    ptr, cells = _rect_cells(nx, ny, tri)
    if jitter > 0.0:
        nodes = _jitter_fast(nodes, xs, ys, nx, ny, jitter, np.random.default_rng(seed), tri)
    kind = {"wall": BCGroup(WALL), "symmetry": BCGroup(SYMMETRY),
            "inlet": BCGroup(INLET, tuple(u_in), rho_inf, internal)}
    groups = [BCGroup(INLET, tuple(u_in), rho_inf, internal),
              BCGroup(OUTLET, tuple(u_in), rho_inf, internal),
              kind[bottom], kind[top]]
    bf, grp, per, sh = _rect_boundary(nx, ny, {"left": 0, "right": 1, "bottom": 2, "top": 3},
                                      Lx=Lx, Ly=Ly)
    return RawMesh(nodes, ptr, cells, bf, grp, groups, per, sh,
                   name=f"channel_{nx}x{ny}", meta=dict(kind="channel", U=float(np.hypot(*u_in))))


def cylinder(nr: int = 256, nt: int = 384, r0: float = 0.5, R: float = 30.0,
             h0: float = 0.005, u_inf=(0.1, 0.0), rho_inf: float = 1.0) -> RawMesh:
    """Body-fitted O-grid around a cylinder of diameter 2*r0 (Section 3.3).

    Radial spacing grows geometrically from h0 at the wall to the far-field
    radius R; the ratio is solved so that nr cells reach R exactly.  Far-field
    edges are outlets where u_inf points out of the domain and inlets elsewhere
    (a tie goes to the inlet)."""
    q = solve_geometric_ratio(h0, nr, R - r0)
    k = np.arange(nr + 1)
    r = r0 + (h0 * k if abs(q - 1) < 1e-14 else h0 * (q ** k - 1.0) / (q - 1.0))
    r[-1] = R
    th = 2.0 * np.pi * np.arange(nt) / nt
    # node (k, m) = k*nt + m
    nodes = np.stack([(r[:, None] * np.cos(th)[None, :]).ravel(),
                      (r[:, None] * np.sin(th)[None, :]).ravel()], axis=1)
    kk, mm = np.meshgrid(np.arange(nr), np.arange(nt), indexing="ij")
    kk = kk.ravel(); mm = mm.ravel(); m1 = (mm + 1) % nt
    # CCW: (r_k, t_m) -> (r_k+1, t_m) -> (r_k+1, t_m+1) -> (r_k, t_m+1)
    cells = np.stack([kk * nt + mm, (kk + 1) * nt + mm, (kk + 1) * nt + m1, kk * nt + m1], axis=1)
    ptr = np.arange(0, 4 * cells.shape[0] + 1, 4, dtype=np.int32)
    groups = [BCGroup(WALL, (0.0, 0.0)),
              BCGroup(INLET, tuple(u_inf), rho_inf, 0),
              BCGroup(OUTLET, tuple(u_inf), rho_inf, 0)]
    bf, grp = [], []
    for m in range(nt):
        bf.append((m, (m + 1) % nt)); grp.append(0)
    for m in range(nt):
        a = nr * nt + m; b = nr * nt + (m + 1) % nt
        # outward direction of the far-field edge: the edge midpoint direction
        # (sign test only; the method's normals are computed by the solvers)
        mx = 0.5 * (nodes[a, 0] + nodes[b, 0]); my = 0.5 * (nodes[a, 1] + nodes[b, 1])
        out = u_inf[0] * mx + u_inf[1] * my
        bf.append((a, b)); grp.append(2 if out > 0.0 else 1)
    return RawMesh(nodes.astype(np.float64), ptr, cells.ravel().astype(np.int32),
                   np.asarray(bf, dtype=np.int32), np.asarray(grp, dtype=np.int32), groups,
                   np.zeros((0, 2), np.int32), np.zeros((0, 2), np.float64),
                   name=f"cylinder_{nr}x{nt}",
                   meta=dict(kind="cylinder", U=float(np.hypot(*u_inf)), D=2 * r0, ratio=q))


def two_cylinders(nr: int = 128, nt: int = 256, spacing: float = 3.0, r0: float = 0.5,
                  half_width: float = 30.0, height: float = 30.0, h0: float = 0.005,
                  u_inf=(0.1, 0.0), rho_inf: float = 1.0) -> RawMesh:
    """Two cylinders side by side (centres (0, +-spacing/2)), two conforming O-blocks.

    The upper block maps the annulus from its cylinder out to the boundary of
    the half-domain rectangle [-W, W] x [0, H] along rays, with a per-ray
    geometric stretching from h0 at the wall; the lower block is its mirror
    image.  The blocks share the nodes on y = 0, which becomes an interior
    interface.  Far-field edges are inlets/outlets by the sign of u_inf.n."""
    W, H = half_width, height
    yc = spacing / 2.0
    th = 2.0 * np.pi * np.arange(nt) / nt - np.pi / 2.0     # start pointing down (towards y = 0)
    # boundary point of the rectangle [-W,W]x[0,H] hit by the ray from (0,yc) at angle th
    bx = np.empty(nt); by = np.empty(nt)
    for m, t in enumerate(th):
        dx, dy = math.cos(t), math.sin(t)
        cand = []
        if dx > 1e-15: cand.append((W) / dx)
        if dx < -1e-15: cand.append((-W) / dx)
        if dy > 1e-15: cand.append((H - yc) / dy)
        if dy < -1e-15: cand.append((0.0 - yc) / dy)
        s = min(c for c in cand if c > 0)
        bx[m] = s * dx; by[m] = yc + s * dy
        if abs(by[m]) < 1e-9:
            by[m] = 0.0
        if abs(abs(bx[m]) - W) < 1e-9:
            bx[m] = math.copysign(W, bx[m])
        if abs(by[m] - H) < 1e-9:
            by[m] = H
    upper = np.zeros((nr + 1, nt, 2))
    for m in range(nt):
        wx = r0 * math.cos(th[m]); wy = yc + r0 * math.sin(th[m])
        L = math.hypot(bx[m] - wx, by[m] - wy)
        q = solve_geometric_ratio(h0, nr, L)
        k = np.arange(nr + 1)
        s = h0 * (q ** k - 1.0) / (q - 1.0)
        s[-1] = L
        upper[:, m, 0] = wx + (bx[m] - wx) * s / L
        upper[:, m, 1] = wy + (by[m] - wy) * s / L
        upper[nr, m] = (bx[m], by[m])
    # the rays that end on y = 0 in the upper block: outer nodes with by == 0
    on_axis = np.abs(upper[nr, :, 1]) < 1e-12
    # lower block is the mirror image (y -> -y); mirror reverses orientation, so
    # index its circumferential direction backwards to keep CCW cells
    lower = upper.copy(); lower[..., 1] *= -1.0
    lower = lower[:, ::-1, :]
    on_axis_lower = on_axis[::-1]
    nU = (nr + 1) * nt
    node_list = [upper.reshape(-1, 2)]
    # lower nodes: reuse upper outer nodes on y = 0
    lower_ids = np.arange(nU, nU + (nr + 1) * nt).reshape(nr + 1, nt)
    # map the mirrored outer axis nodes to the upper ones
    up_outer_idx = {}
    for m in range(nt):
        if on_axis[m]:
            up_outer_idx[round(upper[nr, m, 0], 12)] = nr * nt + m
    new_lower = lower.reshape(-1, 2).copy()
    remap = np.full((nr + 1) * nt, -1, dtype=np.int64)
    for m in range(nt):
        if on_axis_lower[m]:
            key = round(lower[nr, m, 0], 12)
            remap[nr * nt + m] = up_outer_idx[key]
    keep = remap < 0
    fresh = np.cumsum(keep) - 1 + nU
    lower_ids = np.where(keep, fresh, remap).reshape(nr + 1, nt)
    node_list.append(new_lower[keep])
    nodes = np.concatenate(node_list, axis=0)
    upper_ids = np.arange(nU).reshape(nr + 1, nt)

    def block_cells(ids):
        kk, mm = np.meshgrid(np.arange(nr), np.arange(nt), indexing="ij")
        kk = kk.ravel(); mm = mm.ravel(); m1 = (mm + 1) % nt
        return np.stack([ids[kk, mm], ids[kk + 1, mm], ids[kk + 1, m1], ids[kk, m1]], axis=1)

    cells = np.concatenate([block_cells(upper_ids), block_cells(lower_ids)], axis=0)
    ptr = np.arange(0, 4 * cells.shape[0] + 1, 4, dtype=np.int32)
    groups = [BCGroup(WALL, (0.0, 0.0)),
              BCGroup(INLET, tuple(u_inf), rho_inf, 0),
              BCGroup(OUTLET, tuple(u_inf), rho_inf, 0)]
    bf, grp = [], []
    for ids, axis_mask in ((upper_ids, on_axis), (lower_ids, on_axis_lower)):
        for m in range(nt):
            bf.append((ids[0, m], ids[0, (m + 1) % nt])); grp.append(0)
        for m in range(nt):
            m1 = (m + 1) % nt
            if axis_mask[m] and axis_mask[m1]:
                continue                      # interior interface y = 0
            a, b = ids[nr, m], ids[nr, m1]
            mx = 0.5 * (nodes[a, 0] + nodes[b, 0])
            # outward direction of a rectangle side: by which side the edge lies on
            if abs(abs(mx) - W) < 1e-9 and abs(nodes[a, 0] - nodes[b, 0]) < 1e-9:
                nvec = (math.copysign(1.0, mx), 0.0)
            else:
                nvec = (0.0, math.copysign(1.0, 0.5 * (nodes[a, 1] + nodes[b, 1])))
            out = u_inf[0] * nvec[0] + u_inf[1] * nvec[1]
            bf.append((a, b)); grp.append(2 if out > 0.0 else 1)
    return RawMesh(nodes.astype(np.float64), ptr, cells.ravel().astype(np.int32),
                   np.asarray(bf, dtype=np.int32), np.asarray(grp, dtype=np.int32), groups,
                   np.zeros((0, 2), np.int32), np.zeros((0, 2), np.float64),
                   name=f"two_cylinders_{nr}x{nt}x2",
                   meta=dict(kind="two_cylinders", U=float(np.hypot(*u_inf)), D=2 * r0))


def cell_count_cavity(n: int) -> int:
    return 2 * n * n


def streaming_cavity(n: int = 2048, seed: int = 0, lid_u: float = 0.1) -> RawMesh:
    """The 100 x 100 cavity's tanh mapping (growth 1.08 at 100 cells) refined to
    n x n, split and jittered like it: 2 n^2 triangles, far larger than the
    on-chip caches (the bandwidth-roofline workload)."""
    return cavity(n=n, beta=tanh_beta(100, 1.08), jitter=0.2, seed=seed, lid_u=lid_u)


def random_instance(rng: np.random.Generator, n_cells: int, kind: Optional[str] = None):
    """One seeded instance for batched/served workloads: a jittered-triangle
    cavity or an O-grid cylinder of about n_cells cells.  Returns (mesh, Re)."""
    if kind is None:
        kind = "cavity" if rng.random() < 0.5 else "cylinder"
    Re = float(rng.uniform(100.0, 3000.0))
    if kind == "cavity":
        n = max(4, int(round(math.sqrt(n_cells / 2.0))))
        m = cavity(n=n, ratio=1.08 if n >= 20 else 1.0, jitter=0.2, seed=int(rng.integers(1 << 30)))
    elif kind == "cylinder":
        nr = max(4, int(round(math.sqrt(n_cells / 1.5))))
        nt = int(round(1.5 * nr))
        m = cylinder(nr=nr, nt=nt, h0=min(0.005, 29.5 / nr / 2))
    else:
        nr = max(4, int(round(math.sqrt(n_cells / 4.0))))
        m = two_cylinders(nr=nr, nt=2 * nr, h0=min(0.005, 25.0 / nr / 2))
    return m, Re, kind


def hybrid(n: int = 12, jitter: float = 0.15, seed: int = 0, lid_u: float = 0.1) -> RawMesh:
    """Mixed triangle/quad cavity: the lower half of an n x n grid stays quads,
    the upper half is split into triangles (a quad layer under a triangle
    region, like the paper's hybrid cylinder meshes, Section 3.3)."""
    xs = np.linspace(0.0, 1.0, n + 1); ys = xs.copy()
    nodes = _structured_nodes(xs, ys)
    nx1 = n + 1
    ptr = [0]; cells = []
    for j in range(n):
        for i in range(n):
            a, b = _nid(i, j, nx1), _nid(i + 1, j, nx1)
            c, d = _nid(i + 1, j + 1, nx1), _nid(i, j + 1, nx1)
            if j < n // 2:
                cells.extend([a, b, c, d]); ptr.append(len(cells))
            else:
                cells.extend([a, b, c]); ptr.append(len(cells))
                cells.extend([a, c, d]); ptr.append(len(cells))
    if jitter > 0.0:
        # quads and triangles share corner nodes: jitter-check both shapes
        P = nodes.reshape(n + 1, nx1, 2)
        rng = np.random.default_rng(seed)
        base = P.copy()
        for _ in range(40):
            cand = base.copy()
            cand[1:n, 1:n, 0] += rng.uniform(-jitter, jitter, (n - 1, n - 1)) / n
            cand[1:n, 1:n, 1] += rng.uniform(-jitter, jitter, (n - 1, n - 1)) / n
            if not (_bad_nodes(cand, n, n, True).any() or _bad_nodes(cand, n, n, False).any()):
                P = cand
                break
        nodes = P.reshape(-1, 2)
    groups = [BCGroup(WALL, (0.0, 0.0)), BCGroup(WALL, (lid_u, 0.0))]
    bf, grp, per, sh = _rect_boundary(n, n, {"bottom": 0, "right": 0, "left": 0, "top": 1})
    return RawMesh(nodes.astype(np.float64), np.asarray(ptr, np.int32), np.asarray(cells, np.int32),
                   bf, grp, groups, per, sh, name=f"hybrid_{n}", meta=dict(kind="hybrid", U=lid_u))
