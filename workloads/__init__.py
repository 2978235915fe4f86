"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module produces geometry and topology only: particle meshes, their edge
tables, lattice layouts, incidence descriptions and seeded random vectors.  It
holds none of the method's arithmetic (no basis functions, no Green's
functions, no quadrature, no static modes); both the oracle and the library
build those from these inputs on their own.

Units: lengths in wavelengths of the background medium (lambda = 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "icosphere", "cylinder", "edge_table", "check_closed_mesh", "lattice",
    "Incidence", "normal_incidence_x", "c3_incidences", "tilted_incidences",
    "random_complex", "Workload", "workload", "lens_diameters",
]


# ---------------------------------------------------------------- meshes --

def _orient_outward(verts: np.ndarray, tris: np.ndarray) -> np.ndarray:
    """Flip triangles of a star-shaped (about the origin) mesh so that the
    right-hand normal points away from the origin."""
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    nrm = np.cross(v1 - v0, v2 - v0)
    cen = (v0 + v1 + v2) / 3.0
    flip = np.einsum("ij,ij->i", nrm, cen) < 0
    out = tris.copy()
    out[flip] = out[flip][:, [0, 2, 1]]
    return out


def icosphere(radius: float, subdivisions: int = 2):
    """Icosahedron refined by 4-to-1 splits with vertices pushed onto the
    sphere.  subdivisions=2 gives V=162, F=320, E=480.  The base icosahedron
    uses the vertices (0, +-1, +-phi) and cyclic permutations, so the mesh is
    symmetric under the three coordinate mirrors."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    base = []
    for a in (-1.0, 1.0):
        for b in (-phi, phi):
            base += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    verts = np.array(base, dtype=np.float64)
    # faces = triples of mutually adjacent vertices (edge length 2)
    n = len(verts)
    d = np.linalg.norm(verts[:, None, :] - verts[None, :, :], axis=-1)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    tris = np.array(faces, dtype=np.int64)
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    for _ in range(subdivisions):
        vlist = [tuple(v) for v in verts]
        mid_cache: dict[tuple[int, int], int] = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid_cache:
                m = (np.asarray(vlist[a]) + np.asarray(vlist[b])) / 2.0
                m /= np.linalg.norm(m)
                vlist.append(tuple(m))
                mid_cache[key] = len(vlist) - 1
            return mid_cache[key]

        new = []
        for a, b, c in tris:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        verts = np.array(vlist, dtype=np.float64)
        tris = np.array(new, dtype=np.int64)
    tris = _orient_outward(verts, tris)
    return verts * radius, tris.astype(np.int32)


def cylinder(diameter: float, height: float, n_az: int = 20, n_ax: int = 8,
             n_rings: int = 3, jitter: float = 0.01, seed: int = 2407):
    """Closed cylinder about the z axis, centred at the origin.

    Side: n_az x n_ax quads split into triangles; each cap: a centre vertex
    and n_rings inner rings of n_az vertices plus the rim.  The defaults give
    V=302, F=600, E=900.  Every vertex coordinate then receives
    U(-jitter, jitter) * diameter from a generator seeded with ``seed``; the
    orientation is fixed on the unjittered template."""
    R = diameter / 2.0
    ang = 2.0 * np.pi * np.arange(n_az) / n_az
    verts = []
    # side rings k = 0..n_ax (k=0 bottom rim, k=n_ax top rim)
    for k in range(n_ax + 1):
        z = -height / 2.0 + height * k / n_ax
        for a in ang:
            verts.append((R * math.cos(a), R * math.sin(a), z))
    side = lambda k, i: k * n_az + (i % n_az)
    tris = []
    for k in range(n_ax):
        for i in range(n_az):
            a, b = side(k, i), side(k, i + 1)
            c, d = side(k + 1, i + 1), side(k + 1, i)
            tris += [(a, b, c), (a, c, d)]
    # caps
    for top in (False, True):
        z = height / 2.0 if top else -height / 2.0
        rim_ring = n_ax if top else 0
        base = len(verts)
        verts.append((0.0, 0.0, z))
        centre = base
        ring_idx = []
        for r in range(1, n_rings + 1):
            rr = R * r / (n_rings + 1)
            start = len(verts)
            for a in ang:
                verts.append((rr * math.cos(a), rr * math.sin(a), z))
            ring_idx.append([start + i for i in range(n_az)])
        ring_idx.append([side(rim_ring, i) for i in range(n_az)])
        inner = ring_idx[0]
        for i in range(n_az):
            tris.append((centre, inner[i], inner[(i + 1) % n_az]))
        for r in range(n_rings):
            A, B = ring_idx[r], ring_idx[r + 1]
            for i in range(n_az):
                j = (i + 1) % n_az
                tris += [(A[i], B[i], B[j]), (A[i], B[j], A[j])]
    verts = np.array(verts, dtype=np.float64)
    tris = _orient_outward(verts, np.array(tris, dtype=np.int64))
    if jitter:
        rng = np.random.default_rng(seed)
        verts = verts + rng.uniform(-jitter, jitter, size=verts.shape) * diameter
    return verts, tris.astype(np.int32)


def edge_table(tris: np.ndarray) -> np.ndarray:
    """Edge table [ne][4] = (v0, v1, t_plus, t_minus) of a closed oriented
    triangle mesh.  Edges are sorted by (v0, v1) with v0 < v1; t_plus is the
    triangle whose counter-clockwise vertex order runs v0 -> v1, t_minus the
    triangle that runs v1 -> v0."""
    owners: dict[tuple[int, int], list[int]] = {}
    for t, (a, b, c) in enumerate(np.asarray(tris)):
        for u, v in ((a, b), (b, c), (c, a)):
            owners.setdefault((int(u), int(v)), []).append(t)
    edges = []
    for (u, v), ts in owners.items():
        if u < v:
            back = owners.get((v, u))
            if len(ts) != 1 or back is None or len(back) != 1:
                raise ValueError("mesh is not a closed oriented 2-manifold")
            edges.append((u, v, ts[0], back[0]))
    edges.sort()
    return np.array(edges, dtype=np.int32)


def check_closed_mesh(verts: np.ndarray, tris: np.ndarray) -> dict:
    """Euler characteristic, manifoldness and signed volume of a mesh."""
    e = edge_table(tris)
    v0, v1, v2 = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    vol = np.einsum("ij,ij->i", v0, np.cross(v1, v2)).sum() / 6.0
    return {"V": len(verts), "F": len(tris), "E": len(e),
            "euler": len(verts) - len(e) + len(tris), "volume": vol}


# --------------------------------------------------------------- layouts --

def lattice(nx: int, ny: int, pitch: float = 0.5) -> np.ndarray:
    """Centres of an nx x ny square lattice in the z=0 plane, row-major in
    (y, x), with the (0, 0) site at the origin."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    c = np.zeros((ny * nx, 3))
    c[:, 0] = ix.ravel() * pitch
    c[:, 1] = iy.ravel() * pitch
    return c


def lens_diameters(nx: int, ny: int, pitch: float, focal: float,
                   dmin: float = 0.12, dmax: float = 0.40, noise: float = 0.01,
                   n_bins: int = 32, seed: int = 21724):
    """Diameter map of a synthetic metalens: the hyperbolic focusing phase
    2*pi*(f - sqrt(f^2 + x^2 + y^2)) mod 2*pi (x, y measured from the array
    centre) mapped linearly to [dmin, dmax], plus U(-noise, noise) seeded
    noise, clipped and binned into n_bins uniform classes.  Returns
    (class_id per site, bin-centre diameter per class)."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = (ix.ravel() - (nx - 1) / 2.0) * pitch
    y = (iy.ravel() - (ny - 1) / 2.0) * pitch
    ph = np.mod(2 * np.pi * (focal - np.sqrt(focal ** 2 + x ** 2 + y ** 2)), 2 * np.pi)
    d = dmin + (dmax - dmin) * ph / (2 * np.pi)
    d = d + np.random.default_rng(seed).uniform(-noise, noise, size=d.shape)
    d = np.clip(d, dmin, dmax)
    edges = np.linspace(dmin, dmax, n_bins + 1)
    cls = np.clip(np.searchsorted(edges, d, side="right") - 1, 0, n_bins - 1)
    centres = 0.5 * (edges[:-1] + edges[1:])
    return cls.astype(np.int32), centres


# ------------------------------------------------------------- incidence --

@dataclass
class Incidence:
    """Plane wave E = pol * exp(-j k khat . r) in the background medium."""
    khat: np.ndarray      # [3] unit propagation direction
    pol: np.ndarray       # [3] complex polarisation, orthogonal to khat

    def as_arrays(self):
        return np.asarray(self.khat, float), np.asarray(self.pol, complex)


def normal_incidence_x() -> Incidence:
    return Incidence(np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0], complex))


def _angles_incidence(theta, phi, te):
    st, ct, sp, cp = math.sin(theta), math.cos(theta), math.sin(phi), math.cos(phi)
    khat = np.array([st * cp, st * sp, ct])
    th_hat = np.array([ct * cp, ct * sp, -st])
    ph_hat = np.array([-sp, cp, 0.0])
    pol = ph_hat if te else th_hat
    return Incidence(khat, pol.astype(complex))


def c3_incidences():
    """64 incidences: polar 5*i deg (i=0..7) x azimuth 45*j deg (j=0..7);
    TE (E along phi-hat) when i+j is even, TM (E along theta-hat) when odd."""
    out = []
    for i in range(8):
        for j in range(8):
            out.append(_angles_incidence(math.radians(5.0 * i),
                                         math.radians(45.0 * j), (i + j) % 2 == 0))
    return out


def tilted_incidences(n: int, max_deg: float):
    """n x-polarised incidences in the xz plane, polar angle max_deg*i/(n-1)."""
    out = []
    for i in range(n):
        th = math.radians(max_deg * i / max(n - 1, 1))
        out.append(_angles_incidence(th, 0.0, False))
    return out


def random_complex(shape, seed: int = 1) -> np.ndarray:
    """Complex standard-normal array (real and imaginary parts N(0, 1/2))."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


# ------------------------------------------------------------- workloads --

@dataclass
class Workload:
    """A particle array: per-class meshes, centres, class ids and material."""
    name: str
    centers: np.ndarray                 # [P][3]
    class_id: np.ndarray                # [P] int32
    meshes: list                        # per class (verts, tris, edges)
    eps_r: complex                      # particle relative permittivity
    n_perp: int
    n_par: int
    leaf_size: float = 0.5
    incidences: list = field(default_factory=list)

    @property
    def n_particles(self):
        return len(self.centers)

    @property
    def n_unknowns(self):
        return 2 * (self.n_perp + self.n_par) * self.n_particles


def _mesh_with_edges(vt):
    v, t = vt
    return (v, t, edge_table(t))


def workload(name: str, nx: int | None = None, ny: int | None = None) -> Workload:
    """Named synthetic workloads.

    ``c1``: 4x4 dielectric spheres (radius 0.15, eps 4), icosphere with 320
    triangles, 20+20 static modes, pitch 0.5, normal x-polarised incidence.
    ``c2``: 40x40 dielectric cylinders (D 0.3, H 0.6, eps 6.25), 600-triangle
    jittered mesh (seed 2407), 15+15 modes, pitch 0.5.  ``nx``/``ny`` shrink
    the array for small parity cases.  ``c3`` is c2 with 64 incidences.
    ``c4``: 80x80 metalens of the same cylinders (H 0.6, eps 6.25) with
    diameters from the focusing profile of ``lens_diameters`` (focal length
    20), 32 diameter classes, one mesh per class (jitter seed 2407 + class).
    ``c5``: the 200x200 lens (focal length 50) with 16 incidences tilted up
    to 20 degrees.  ``nx``/``ny`` give a smaller lens of the same recipe.
    ``c5_sparse``: 18 particles of the c5 lens at the sites SPARSE_SITES,
    spanning its full 200 x 200 extent (all seven tree levels)."""
    name = name.lower()
    if name == "c1":
        nx, ny = nx or 4, ny or 4
        mesh = _mesh_with_edges(icosphere(0.15, 2))
        return Workload("c1", lattice(nx, ny, 0.5), np.zeros(nx * ny, np.int32),
                        [mesh], 4.0 + 0j, 20, 20, 0.5, [normal_incidence_x()])
    if name in ("c2", "c3"):
        nx, ny = nx or 40, ny or 40
        mesh = _mesh_with_edges(cylinder(0.3, 0.6))
        inc = [normal_incidence_x()] if name == "c2" else c3_incidences()
        return Workload(name, lattice(nx, ny, 0.5), np.zeros(nx * ny, np.int32),
                        [mesh], 6.25 + 0j, 15, 15, 0.5, inc)
    if name in ("c4", "c5"):
        # metalens: diameters from the hyperbolic focusing profile, 32 classes
        nx = nx or (80 if name == "c4" else 200)
        ny = ny or nx
        focal = 20.0 if name == "c4" else 50.0
        cls, dia = lens_diameters(nx, ny, 0.5, focal)
        meshes = [_mesh_with_edges(cylinder(float(d), 0.6, seed=2407 + c)) for c, d in enumerate(dia)]
        inc = [normal_incidence_x()] if name == "c4" else tilted_incidences(16, 20.0)
        return Workload(name, lattice(nx, ny, 0.5), cls, meshes, 6.25 + 0j, 15, 15, 0.5, inc)
    if name == "c5_sparse":
        # 18 particles of the 200x200 lens at sites spread over the whole
        # aperture (the corners fix the extent), so that particle pairs are
        # separated at every level of its tree; each keeps the class the
        # lens gives its site
        cls, dia = lens_diameters(200, 200, 0.5, 50.0)
        meshes = [_mesh_with_edges(cylinder(float(d), 0.6, seed=2407 + c)) for c, d in enumerate(dia)]
        sites = np.array(SPARSE_SITES)
        cen = np.zeros((len(sites), 3))
        cen[:, :2] = 0.5 * sites
        return Workload(name, cen, cls[sites[:, 1] * 200 + sites[:, 0]], meshes, 6.25 + 0j, 15, 15, 0.5,
                        tilted_incidences(2, 20.0))
    raise ValueError(f"unknown workload {name}")


# (ix, iy) lattice sites of the sparse full-extent lens: pairs adjacent (near
# field) and separated at each of the seven levels of the 200 x 200 tree
SPARSE_SITES = [(0, 0), (2, 0), (0, 5), (9, 3), (20, 1), (37, 12), (70, 40), (120, 30), (199, 199), (150, 180),
                (100, 100), (101, 100), (100, 101), (60, 140), (10, 190), (190, 10), (130, 130), (103, 98)]
