"""Seeded synthetic workloads for the flip-free ADMM solver.

This module only builds inputs (source vertices V, elements T, pins and an
initial map).  It holds none of the method's arithmetic, so both the GPU
path and the CPU oracle can be driven from it.

The paper measures on named meshes and on a UV-mapping dataset that are not
available here; the generators below are synthetic stand-ins of the same
kind (height-field and sphere-cap UV charts, a twisted tet cube, a 2D disk
for deformation), sized like the paper's range of 3.6k to 2.4M elements
(runtime table of the comparison section).

Every generator draws from ``numpy.random.default_rng([210705200, c])``
(PCG64) for workload number ``c``, in the order stated in its docstring.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

SEED_BASE = 210705200

SYMMETRIC_DIRICHLET = 0
SYMMETRIC_GRADIENT = 1


@dataclass
class Workload:
    """One synthetic problem instance.

    V : (n, d_in) float64 source vertices.
    T : (m, d+1) int32 elements, positively oriented.
    pinned_idx : (p,) int32, pinned_pos : (p, d) float64 pinned targets.
    x0 : (n, d) float64 initial map.  Its pinned rows need not equal
         ``pinned_pos`` (the deformation workloads start from x0 = V);
         the first W-step puts them there.
    """
    name: str
    V: np.ndarray
    T: np.ndarray
    energy: int
    rho: float
    pinned_idx: np.ndarray
    pinned_pos: np.ndarray
    x0: np.ndarray
    iters: int
    meta: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return self.T.shape[1] - 1

    @property
    def n(self) -> int:
        return self.V.shape[0]

    @property
    def m(self) -> int:
        return self.T.shape[0]


def rng_for(c: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, c])


# ----------------------------------------------------------------------------
# grids and disks
# ----------------------------------------------------------------------------

def grid_triangles(k: int) -> np.ndarray:
    """Triangles of a (k+1) x (k+1) vertex grid, vertex (i, j) -> j*(k+1)+i.

    Each cell with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) gives
    the counter-clockwise triangles (a, b, c) and (a, c, d)."""
    s = k + 1
    i, j = np.meshgrid(np.arange(k), np.arange(k), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    a = j * s + i
    b = j * s + i + 1
    c = (j + 1) * s + i + 1
    d = (j + 1) * s + i
    # cell-major: both triangles of a cell are adjacent in the list
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    T = np.empty((2 * k * k, 3), dtype=np.int64)
    T[0::2] = t1
    T[1::2] = t2
    return T.astype(np.int32)


def hex_disk(R: int):
    """Hexagonal-ring disk: a centre vertex and rings r = 1..R with 6r vertices
    at angles 2*pi*t/(6r).  Returns (ring, t, T) with T counter-clockwise in the
    (r cos phi, r sin phi) plane; m = 6 R^2, n = 1 + 3 R (R+1)."""
    ring = [np.zeros(1, dtype=np.int64)]
    tt = [np.zeros(1, dtype=np.int64)]
    start = [0]
    nxt = 1
    for r in range(1, R + 1):
        start.append(nxt)
        ring.append(np.full(6 * r, r, dtype=np.int64))
        tt.append(np.arange(6 * r, dtype=np.int64))
        nxt += 6 * r
    ring = np.concatenate(ring)
    tt = np.concatenate(tt)
    tris = []
    for r in range(1, R + 1):
        o0 = start[r]
        no = 6 * r
        if r == 1:
            for k in range(6):
                tris.append((0, o0 + k, o0 + (k + 1) % no))
            continue
        i0 = start[r - 1]
        ni = 6 * (r - 1)
        for s in range(6):
            for k in range(r):
                a = o0 + (s * r + k) % no
                b = o0 + (s * r + k + 1) % no
                c = i0 + (s * (r - 1) + k) % ni
                tris.append((c, a, b))
            for k in range(r - 1):
                a = i0 + (s * (r - 1) + k) % ni
                b = o0 + (s * r + k + 1) % no
                c = i0 + (s * (r - 1) + k + 1) % ni
                tris.append((a, b, c))
    T = np.asarray(tris, dtype=np.int64)
    # orient counter-clockwise in the flat disk
    phi = 2.0 * np.pi * tt / np.maximum(6 * ring, 1)
    P = np.stack([ring * np.cos(phi), ring * np.sin(phi)], axis=1).astype(np.float64)
    e1 = P[T[:, 1]] - P[T[:, 0]]
    e2 = P[T[:, 2]] - P[T[:, 0]]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    neg = det < 0
    T[neg, 1], T[neg, 2] = T[neg, 2].copy(), T[neg, 1].copy()
    return ring, tt, T.astype(np.int32)


def kuhn_cube(k: int):
    """(k+1)^3 lattice on [0,1]^3 with vertex (i,j,l) -> (l*(k+1)+j)*(k+1)+i; each
    cell is split into the 6 Kuhn tetrahedra 000 -> e_s1 -> e_s1+e_s2 -> 111
    (one per axis permutation), oriented to positive volume.  m = 6 k^3."""
    s = k + 1
    ii, jj, ll = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    V = np.zeros((s ** 3, 3))
    idx = (ll * s + jj) * s + ii
    V[idx.ravel(), 0] = ii.ravel() / k
    V[idx.ravel(), 1] = jj.ravel() / k
    V[idx.ravel(), 2] = ll.ravel() / k
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    ci, cj, cl = np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij")
    # cell order: l slowest, then j, then i (matches the vertex numbering)
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    cl = cl.transpose(2, 1, 0).ravel()

    def vid(a, b, c):
        return (c * s + b) * s + a

    tets = []
    for p in perms:
        off = np.zeros(3, dtype=np.int64)
        verts = [vid(ci, cj, cl)]
        for ax in p[:2]:
            off[ax] += 1
            verts.append(vid(ci + off[0], cj + off[1], cl + off[2]))
        verts.append(vid(ci + 1, cj + 1, cl + 1))
        tets.append(np.stack(verts, axis=1))
    T = np.stack(tets, axis=1).reshape(-1, 4)  # cell-major, 6 tets per cell
    e = V[T[:, 1:]] - V[T[:, [0]]]
    det = np.linalg.det(e)
    neg = det < 0
    T[neg, 2], T[neg, 3] = T[neg, 3].copy(), T[neg, 2].copy()
    return V, T.astype(np.int32)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def height_field_uv(grid: int = 32, sigma: float = 0.02, seed_c: int = 1,
                    rho: float = 10.0, iters: int = 200,
                    energy: int = SYMMETRIC_DIRICHLET) -> Workload:
    """Height-field UV chart (1,922 triangles at grid=32).

    Vertex (i, j), i, j in 0..grid-1, index j*grid+i, source
    V = (x, y, 0.3 sin(3x) cos(2y)) with x = i/(grid-1), y = j/(grid-1).
    Draws: x0 = (x, y) + N(0, sigma^2) per coordinate, vertex by vertex.
    Pins: vertex 0 at (0, 0) and the last vertex at (1, 1), noise-free."""
    k = grid - 1
    T = grid_triangles(k)
    i, j = np.meshgrid(np.arange(grid), np.arange(grid), indexing="xy")
    x = (i.ravel() / k).astype(np.float64)
    y = (j.ravel() / k).astype(np.float64)
    V = np.stack([x, y, 0.3 * np.sin(3 * x) * np.cos(2 * y)], axis=1)
    rng = rng_for(seed_c)
    x0 = np.stack([x, y], axis=1) + rng.normal(0.0, sigma, size=(grid * grid, 2))
    pins = np.array([0, grid * grid - 1], dtype=np.int32)
    ppos = np.array([[0.0, 0.0], [1.0, 1.0]])
    x0[pins] = ppos
    return Workload(f"height_field_uv_{grid}", V, T, energy, rho, pins, ppos, x0, iters,
                    {"grid": grid, "sigma": sigma})


def sphere_cap_uv(R: int = 289, seed_c: int = 2, rho: float = 10.0, iters: int = 500,
                  energy: int = SYMMETRIC_GRADIENT) -> Workload:
    """Noisy sphere cap, geodesic radius 1.2 rad, UV-mapped with the symmetric
    gradient energy (501,126 triangles at R=289).

    A hexagonal-ring disk of R rings; ring fraction s = r/R maps to polar
    angle theta = 1.2 s and azimuth phi = 2 pi t/(6r).
    Draws: radial noise N(0, 0.01^2) per vertex, then the initial-map noise
    N(0, (0.2*1.2/R)^2) per coordinate, vertex by vertex.
    x0 = theta (cos phi, sin phi) + noise (an azimuthal-equidistant disk,
    convex boundary, flip-free before the noise), translated so that
    x0[0] = 0; vertex 0 is the single pin (the paper fixes the first vertex
    when a UV map has no constraints)."""
    ring, tt, T = hex_disk(R)
    n = ring.shape[0]
    theta = 1.2 * ring / R
    phi = 2.0 * np.pi * tt / np.maximum(6 * ring, 1)
    rng = rng_for(seed_c)
    radial = 1.0 + rng.normal(0.0, 0.01, size=n)
    V = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)],
                 axis=1) * radial[:, None]
    x0 = np.stack([theta * np.cos(phi), theta * np.sin(phi)], axis=1)
    x0 = x0 + rng.normal(0.0, 0.2 * 1.2 / R, size=(n, 2))
    x0 = x0 - x0[0]
    pins = np.array([0], dtype=np.int32)
    ppos = x0[pins].copy()
    return Workload(f"sphere_cap_uv_R{R}", V, T, energy, rho, pins, ppos, x0, iters, {"R": R})


def twisted_cube(k: int = 64, twist_deg: float = 45.0, lift: float = 0.3,
                 rho: float = 10.0, iters: int = 300,
                 energy: int = SYMMETRIC_DIRICHLET) -> Workload:
    """Tet cube deformation (1,572,864 tets, 274,625 vertices at k=64).

    Bottom face (z = 0) pinned at rest; top face (z = 1) rotated by
    ``twist_deg`` about the vertical axis through (0.5, 0.5) and lifted by
    ``lift``.  x0 = V (rest pose).  No random draws."""
    V, T = kuhn_cube(k)
    s = k + 1
    bottom = np.arange(s * s, dtype=np.int64)
    top = np.arange(k * s * s, s * s * s, dtype=np.int64)
    a = math.radians(twist_deg)
    ca, sa = math.cos(a), math.sin(a)
    pt = V[top].copy()
    dx, dy = pt[:, 0] - 0.5, pt[:, 1] - 0.5
    pt[:, 0] = 0.5 + ca * dx - sa * dy
    pt[:, 1] = 0.5 + sa * dx + ca * dy
    pt[:, 2] = pt[:, 2] + lift
    pins = np.concatenate([bottom, top]).astype(np.int32)
    ppos = np.concatenate([V[bottom], pt])
    x0 = V.copy()
    return Workload(f"twisted_cube_{k}", V, T, energy, rho, pins, ppos, x0, iters, {"k": k})


def batched_charts(n_charts: int = 256, seed_c: int = 4, m_lo: float = 200.0,
                   m_hi: float = 50000.0, rho: float = 10.0, iters: int = 200):
    """Many independent height-field charts of uneven size (256 charts by default).

    Per chart j, in order: m_j = exp(U(ln m_lo, ln m_hi)); a_j ~ U(0.1, 0.4);
    b_j, c_j ~ U(1, 4); then the initial-map noise N(0, (0.62/k_j)^2) per
    coordinate, vertex by vertex, with k_j = round(sqrt(m_j/2)) cells per side.
    Energy: symmetric Dirichlet for even j, symmetric gradient for odd j.
    Pins: the two grid corners (0,0) and (1,1)."""
    rng = rng_for(seed_c)
    out = []
    for j in range(n_charts):
        mj = math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))
        aj = rng.uniform(0.1, 0.4)
        bj = rng.uniform(1.0, 4.0)
        cj = rng.uniform(1.0, 4.0)
        k = max(1, int(round(math.sqrt(mj / 2.0))))
        g = k + 1
        T = grid_triangles(k)
        ii, jj = np.meshgrid(np.arange(g), np.arange(g), indexing="xy")
        x = ii.ravel() / k
        y = jj.ravel() / k
        V = np.stack([x, y, aj * np.sin(bj * x) * np.cos(cj * y)], axis=1)
        x0 = np.stack([x, y], axis=1) + rng.normal(0.0, 0.62 / k, size=(g * g, 2))
        pins = np.array([0, g * g - 1], dtype=np.int32)
        ppos = np.array([[0.0, 0.0], [1.0, 1.0]])
        x0[pins] = ppos
        energy = SYMMETRIC_DIRICHLET if j % 2 == 0 else SYMMETRIC_GRADIENT
        out.append(Workload(f"chart_{j}", V, T, energy, rho, pins, ppos, x0, iters,
                            {"k": k, "a": aj, "b": bj, "c": cj}))
    return out


def disk_deformation(R: int = 129, n_handles: int = 16, seed_c: int = 5,
                     rho: float = 10.0, iters: int = 100,
                     energy: int = SYMMETRIC_DIRICHLET) -> Workload:
    """2D disk deformation with displaced handles (99,846 triangles at R=129).

    Planar hexagonal-ring disk of radius 1.  Draws: ``n_handles`` handle
    vertices without replacement, then targets V_h + N(0, 0.1^2) per
    coordinate, handle by handle.  x0 = V."""
    ring, tt, T = hex_disk(R)
    phi = 2.0 * np.pi * tt / np.maximum(6 * ring, 1)
    rr = ring / R
    V = np.stack([rr * np.cos(phi), rr * np.sin(phi)], axis=1)
    rng = rng_for(seed_c)
    handles = np.sort(rng.choice(V.shape[0], size=n_handles, replace=False)).astype(np.int32)
    targets = V[handles] + rng.normal(0.0, 0.1, size=(n_handles, 2))
    x0 = V.copy()
    return Workload(f"disk_deformation_R{R}", V, T, energy, rho, handles, targets, x0, iters,
                    {"R": R})


def flat_grid(grid: int = 8, rho: float = 10.0, energy: int = SYMMETRIC_DIRICHLET) -> Workload:
    """Flat planar grid with x0 = V (a fixed point of the iteration)."""
    k = grid - 1
    T = grid_triangles(k)
    i, j = np.meshgrid(np.arange(grid), np.arange(grid), indexing="xy")
    V = np.stack([i.ravel() / k, j.ravel() / k], axis=1).astype(np.float64)
    pins = np.array([0, grid * grid - 1], dtype=np.int32)
    return Workload(f"flat_grid_{grid}", V, T, energy, rho, pins, V[pins].copy(), V.copy(), 10)


# ----------------------------------------------------------------------------
# fixed boundaries for Tutte initial maps (inputs, not part of the method)
# ----------------------------------------------------------------------------

def boundary_vertices(T) -> np.ndarray:
    """Sorted vertices of the facets that belong to exactly one element."""
    T = np.asarray(T, dtype=np.int64)
    nc = T.shape[1]
    faces = np.concatenate([np.sort(np.delete(T, c, axis=1), axis=1) for c in range(nc)], axis=0)
    uniq, cnt = np.unique(faces, axis=0, return_counts=True)
    return np.unique(uniq[cnt == 1]).astype(np.int32)


def boundary_loop(T) -> np.ndarray:
    """The boundary of a triangulated disk as one closed vertex loop, walked
    along the directed edges of the triangles (counter-clockwise for
    counter-clockwise triangles)."""
    T = np.asarray(T, dtype=np.int64)
    directed = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]], axis=0)
    n = int(T.max()) + 1
    key = directed[:, 0] * n + directed[:, 1]
    rev = directed[:, 1] * n + directed[:, 0]
    bnd = directed[~np.isin(rev, key)]
    if np.unique(bnd[:, 0]).size != bnd.shape[0]:
        raise ValueError("boundary is not a single simple loop")
    nxt = dict(zip(bnd[:, 0].tolist(), bnd[:, 1].tolist()))
    if not nxt:
        raise ValueError("closed surface: no boundary")
    start = min(nxt)
    loop = [start]
    while True:
        v = nxt[loop[-1]]
        if v == start:
            break
        loop.append(v)
        if len(loop) > len(nxt):
            raise ValueError("boundary is not a single simple loop")
    if len(loop) != len(nxt):
        raise ValueError("boundary has several loops")
    return np.asarray(loop, dtype=np.int32)


def circle_boundary(V, T, radius: float = 1.0):
    """The boundary loop of a disk placed on a circle, each vertex at the
    angle of its arc length along the loop in the source mesh.  Returns
    (indices, positions (len, 2))."""
    V = np.asarray(V, dtype=np.float64)
    loop = boundary_loop(T)
    seg = np.linalg.norm(V[np.roll(loop, -1)] - V[loop], axis=1)
    arc = np.concatenate([[0.0], np.cumsum(seg)[:-1]])
    ang = 2.0 * np.pi * arc / seg.sum()
    return loop, radius * np.stack([np.cos(ang), np.sin(ang)], axis=1)


WORKLOADS = {
    "height_field_uv": lambda: height_field_uv(),
    "sphere_cap_uv": lambda: sphere_cap_uv(),
    "twisted_cube": lambda: twisted_cube(),
    "disk_deformation": lambda: disk_deformation(),
}


def unit_tangents(w: Workload, count: int, seed_c: int = 21):
    """``count`` random unit directions over (rest vertices, pinned targets):
    for each, dV ~ N(0, 1) of V's shape, then dp ~ N(0, 1) of the targets'
    shape, both divided by the joint Euclidean norm.  Returns a list of
    (dV, dp)."""
    rng = rng_for(seed_c)
    out = []
    for _ in range(count):
        dV = rng.normal(size=w.V.shape)
        dp = rng.normal(size=w.pinned_pos.shape)
        nrm = math.sqrt(float((dV ** 2).sum() + (dp ** 2).sum()))
        out.append((dV / nrm, dp / nrm))
    return out
