"""Seeded synthetic inputs: meshes, Dirichlet data and request streams.

This module only *generates* inputs.  It holds none of the solver's
arithmetic: no element matrices, no assembly, no Dirichlet lifting and no
Krylov step.  Both the plain CPU oracle and the HIP library consume the arrays
it returns, so the two sides always see identical meshes and boundary data.

Workloads follow the paper's case study (Sect. 2.2): the Laplace equation with
Dirichlet data on the unit square / unit cube, discretised on a regular grid or
on an irregular (here: jittered) simplicial mesh.

Random numbers come from one counter-based generator, SplitMix64 (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
draw ``c`` of stream ``s`` under seed ``seed`` is ``mix(key(seed, s) + (c+1)*G)``
with ``G = 0x9E3779B97F4A7C15``; a uniform double in [0,1) is the top 53 bits
times 2^-53; normals use the Box-Muller transform.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

_G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids: one per kind of draw, so changing one input never shifts another
STREAM_JITTER = 1
STREAM_COEFF = 2
STREAM_NOISE = 3
STREAM_ARRIVAL = 4
STREAM_REQUEST = 5


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
        s = _mix(s + np.uint64(stream) * _G)
        return s[0]


def uniform(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` uniform doubles in [0,1): draws offset..offset+count-1."""
    with np.errstate(over="ignore"):
        c = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = _mix(_key(seed, stream) + c * _G)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, stream: int, count: int) -> np.ndarray:
    """``count`` standard normals (Box-Muller on consecutive uniform pairs)."""
    u = uniform(seed, stream, 2 * count).reshape(count, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
    return r * np.cos(2.0 * math.pi * u[:, 1])


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------

def _tri_area2(p0, p1, p2):
    """Twice the signed area of triangles (arrays of shape [..., 2])."""
    return (p1[..., 0] - p0[..., 0]) * (p2[..., 1] - p0[..., 1]) - \
           (p1[..., 1] - p0[..., 1]) * (p2[..., 0] - p0[..., 0])


def _tet_vol6(p0, p1, p2, p3):
    """Six times the signed volume of tetrahedra (arrays [..., 3])."""
    a = p1 - p0
    b = p2 - p0
    c = p3 - p0
    return (a[..., 0] * (b[..., 1] * c[..., 2] - b[..., 2] * c[..., 1])
            - a[..., 1] * (b[..., 0] * c[..., 2] - b[..., 2] * c[..., 0])
            + a[..., 2] * (b[..., 0] * c[..., 1] - b[..., 1] * c[..., 0]))


class Mesh(dict):
    """dim, coords [nv][dim] f64, cells [nc][dim+1] i32 (positive orientation),
    on_boundary [nv] u8, plus generation metadata."""

    @property
    def dim(self):
        return self["dim"]

    @property
    def nverts(self):
        return self["coords"].shape[0]

    @property
    def ncells(self):
        return self["cells"].shape[0]


def mesh2d(m: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """m x m vertices on [0,1]^2, every cell split into two triangles.

    Vertex (i, j) has index i + m*j and sits at (i, j)/(m-1).  Interior
    vertices move by independent U[-jitter*h, +jitter*h] offsets per
    coordinate (draw 2*v + c).  Each cell (a,b,c,d) = ((i,j),(i+1,j),(i+1,j+1),
    (i,j+1)) is cut along the shorter diagonal; ties (the structured grid) take
    a-c; a cut that would leave a triangle with non-positive area takes the
    other diagonal (a jittered cell with jitter < h/2 is a simple
    quadrilateral, so one of the two cuts is always valid).
    """
    if m < 2:
        raise ValueError("m >= 2 required")
    if not (0.0 <= jitter < 0.5):
        raise ValueError("jitter must lie in [0, 0.5)")
    nv = m * m
    h = 1.0 / (m - 1)
    idx = np.arange(m, dtype=np.float64) / (m - 1)
    coords = np.empty((nv, 2), dtype=np.float64)
    coords[:, 0] = np.tile(idx, m)
    coords[:, 1] = np.repeat(idx, m)
    ii = np.tile(np.arange(m), m)
    jj = np.repeat(np.arange(m), m)
    bnd = (ii == 0) | (ii == m - 1) | (jj == 0) | (jj == m - 1)
    if jitter > 0.0:
        u = uniform(seed, STREAM_JITTER, 2 * nv).reshape(nv, 2)
        d = (2.0 * u - 1.0) * (jitter * h)
        d[bnd] = 0.0
        coords += d
    ci = np.tile(np.arange(m - 1), m - 1)
    cj = np.repeat(np.arange(m - 1), m - 1)
    a = (ci + m * cj).astype(np.int64)
    b = a + 1
    c = a + 1 + m
    dd = a + m
    P = coords
    # option AC: (a,b,c), (a,c,d); option BD: (a,b,d), (b,c,d)
    ac_min = np.minimum(_tri_area2(P[a], P[b], P[c]), _tri_area2(P[a], P[c], P[dd]))
    bd_min = np.minimum(_tri_area2(P[a], P[b], P[dd]), _tri_area2(P[b], P[c], P[dd]))
    lac = ((P[c] - P[a]) ** 2).sum(1)
    lbd = ((P[dd] - P[b]) ** 2).sum(1)
    use_ac = lac <= lbd
    use_ac = np.where(use_ac & (ac_min <= 0.0), False, use_ac)
    use_ac = np.where(~use_ac & (bd_min <= 0.0), True, use_ac)
    t0 = np.where(use_ac[:, None], np.stack([a, b, c], 1), np.stack([a, b, dd], 1))
    t1 = np.where(use_ac[:, None], np.stack([a, c, dd], 1), np.stack([b, c, dd], 1))
    cells = np.empty((2 * len(a), 3), dtype=np.int32)
    cells[0::2] = t0
    cells[1::2] = t1
    ar = _tri_area2(P[cells[:, 0]], P[cells[:, 1]], P[cells[:, 2]])
    if not np.all(ar > 0.0):
        raise RuntimeError("mesh2d produced a non-positive triangle")
    return Mesh(dim=2, coords=coords, cells=cells, on_boundary=bnd.astype(np.uint8),
                m=m, jitter=jitter, seed=seed, n_bd_diag=int((~use_ac).sum()))


KUHN_PERMS = list(itertools.permutations((0, 1, 2)))


def mesh3d(m: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """m^3 vertices on [0,1]^3, every cube cut into the 6 Kuhn tetrahedra.

    Vertex (i, j, l) has index i + m*(j + m*l).  The tetrahedron of axis
    permutation (p0,p1,p2) is v0, v0+e_p0, v0+e_p0+e_p1, v0+(1,1,1); odd
    permutations swap their last two vertices so every tet is positively
    oriented.  Jitter: interior vertices move by U[-jitter*h, jitter*h] per
    coordinate (draw 3*v + c); then, while any tetrahedron has non-positive
    volume, the displacement of every vertex of such a tetrahedron is halved.
    This terminates (zero displacement is the valid structured mesh).
    """
    if m < 2:
        raise ValueError("m >= 2 required")
    if not (0.0 <= jitter < 0.5):
        raise ValueError("jitter must lie in [0, 0.5)")
    nv = m ** 3
    h = 1.0 / (m - 1)
    idx = np.arange(m, dtype=np.float64) / (m - 1)
    coords = np.empty((nv, 3), dtype=np.float64)
    coords[:, 0] = np.tile(idx, m * m)
    coords[:, 1] = np.tile(np.repeat(idx, m), m)
    coords[:, 2] = np.repeat(idx, m * m)
    ii = np.tile(np.arange(m), m * m)
    jj = np.tile(np.repeat(np.arange(m), m), m)
    ll = np.repeat(np.arange(m), m * m)
    bnd = (ii == 0) | (ii == m - 1) | (jj == 0) | (jj == m - 1) | (ll == 0) | (ll == m - 1)
    ci = np.tile(np.arange(m - 1), (m - 1) ** 2)
    cj = np.tile(np.repeat(np.arange(m - 1), m - 1), m - 1)
    cl = np.repeat(np.arange(m - 1), (m - 1) ** 2)
    v0 = (ci + m * (cj + m * cl)).astype(np.int64)
    off = (1, m, m * m)
    allo = 1 + m + m * m
    tets = []
    for p in KUHN_PERMS:
        t = [v0, v0 + off[p[0]], v0 + off[p[0]] + off[p[1]], v0 + allo]
        parity = sum(1 for x in range(3) for y in range(x + 1, 3) if p[x] > p[y]) % 2
        if parity == 1:
            t[2], t[3] = t[3], t[2]
        tets.append(np.stack(t, 1))
    cells = np.stack(tets, 1).reshape(-1, 4).astype(np.int32)
    n_damped = 0
    halvings = 0
    if jitter > 0.0:
        u = uniform(seed, STREAM_JITTER, 3 * nv).reshape(nv, 3)
        disp = (2.0 * u - 1.0) * (jitter * h)
        disp[bnd] = 0.0
        damped = np.zeros(nv, dtype=bool)
        base = coords
        while True:
            X = base + disp
            vol = _tet_vol6(X[cells[:, 0]], X[cells[:, 1]], X[cells[:, 2]], X[cells[:, 3]])
            bad = vol <= 0.0
            if not bad.any():
                break
            vb = np.unique(cells[bad].ravel())
            disp[vb] *= 0.5
            damped[vb] = True
            halvings += 1
            if halvings > 200:
                raise RuntimeError("mesh3d jitter damping did not terminate")
        coords = base + disp
        n_damped = int(damped.sum())
    vol = _tet_vol6(coords[cells[:, 0]], coords[cells[:, 1]], coords[cells[:, 2]], coords[cells[:, 3]])
    if not np.all(vol > 0.0):
        raise RuntimeError("mesh3d produced a non-positive tetrahedron")
    return Mesh(dim=3, coords=coords, cells=cells, on_boundary=bnd.astype(np.uint8),
                m=m, jitter=jitter, seed=seed, n_damped=n_damped, halvings=halvings)


def make_mesh(dim: int, m: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    return mesh2d(m, jitter, seed) if dim == 2 else mesh3d(m, jitter, seed)


# ----------------------------------------------------------------------------
# Dirichlet data: harmonic polynomials up to degree 3
# ----------------------------------------------------------------------------

def _basis2(x, y):
    return [np.ones_like(x), x, y, x * x - y * y, x * y,
            x ** 3 - 3 * x * y * y, 3 * x * x * y - y ** 3]


def _basis3(x, y, z):
    return [np.ones_like(x), x, y, z,
            x * y, y * z, z * x, x * x - y * y, y * y - z * z,
            x * y * z,
            x ** 3 - 3 * x * y * y, 3 * x * x * y - y ** 3,
            y ** 3 - 3 * y * z * z, 3 * y * y * z - z ** 3,
            z ** 3 - 3 * z * x * x, 3 * z * z * x - x ** 3]


NBASIS = {2: 7, 3: 16}
# index of x^2 - y^2 in each basis
IDX_X2_MINUS_Y2 = {2: 3, 3: 7}
IDX_X, IDX_Y = 1, 2


def harmonic_basis(coords: np.ndarray) -> np.ndarray:
    """[n][nbasis] values of the harmonic basis at the given points."""
    coords = np.asarray(coords, dtype=np.float64)
    if coords.shape[1] == 2:
        cols = _basis2(coords[:, 0], coords[:, 1])
    else:
        cols = _basis3(coords[:, 0], coords[:, 1], coords[:, 2])
    return np.stack(cols, 1)


def random_coeffs(dim: int, k: int, seed: int) -> np.ndarray:
    """[nbasis][k] N(0,1) coefficients (column-major draw order)."""
    nb = NBASIS[dim]
    return normal(seed, STREAM_COEFF, nb * k).reshape(k, nb).T.copy()


def fixed_coeffs(dim: int, terms: dict) -> np.ndarray:
    c = np.zeros((NBASIS[dim], 1))
    for i, v in terms.items():
        c[i, 0] = v
    return c


def harmonic_eval(coeffs: np.ndarray, coords: np.ndarray) -> np.ndarray:
    """g[n][k] = sum_b basis_b(x_n) * coeffs[b][k]."""
    return harmonic_basis(coords) @ coeffs


def noise(seed: int, n: int, std: float) -> np.ndarray:
    return std * normal(seed, STREAM_NOISE, n)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

class Workload:
    """A mesh, an element order, k Dirichlet columns and a tolerance.

    ``dirichlet(dof_coords)`` evaluates g at every DOF (public DOF order) of
    whichever side asks: both the oracle and the library pass their own DOF
    coordinates, which agree bit for bit on the same mesh.
    """

    def __init__(self, name, mesh, order, k, tol, coeffs, noise_std=0.0, noise_seed=0,
                 note=""):
        self.name = name
        self.mesh = mesh
        self.order = order
        self.k = k
        self.tol = tol
        self.coeffs = coeffs
        self.noise_std = noise_std
        self.noise_seed = noise_seed
        self.note = note

    def dirichlet(self, dof_coords: np.ndarray) -> np.ndarray:
        g = harmonic_eval(self.coeffs, dof_coords)
        if self.noise_std > 0.0:
            g = g + noise(self.noise_seed, g.shape[0] * g.shape[1], self.noise_std).reshape(g.shape)
        return np.ascontiguousarray(g)


def c1(m: int = 64) -> Workload:
    """64x64 structured 2D P1, g = 1 + 2x - 3y, tol 1e-10."""
    mesh = mesh2d(m)
    co = fixed_coeffs(2, {0: 1.0, IDX_X: 2.0, IDX_Y: -3.0})
    return Workload("c1_2d_p1_64", mesh, 1, 1, 1e-10, co)


def c2(m: int = 1024, seed: int = 1, data_seed: int = 2) -> Workload:
    """1024^2 2D P1, jitter 0.3h, g = x^2 - y^2 + N(0, 0.01^2) noise, tol 1e-8."""
    mesh = mesh2d(m, 0.3, seed)
    co = fixed_coeffs(2, {IDX_X2_MINUS_Y2[2]: 1.0})
    return Workload("c2_2d_p1_jit_%d" % m, mesh, 1, 1, 1e-8, co, noise_std=0.01,
                    noise_seed=data_seed)


def c3(m: int = 128, k: int = 32, seed: int = 3) -> Workload:
    """128^3 structured Kuhn P1, k=32 random harmonic cubics, tol 1e-8."""
    mesh = mesh3d(m)
    return Workload("c3_3d_p1_%d_k%d" % (m, k), mesh, 1, k, 1e-8, random_coeffs(3, k, seed))


def c4(m: int = 513, k: int = 8, seed: int = 4, data_seed: int = 5) -> Workload:
    """P2 on 513^2 vertices (512^2 cells), jitter 0.25h; column 0 = x^2 - y^2,
    columns 1..k-1 random harmonic data; tol 1e-8."""
    mesh = mesh2d(m, 0.25, seed)
    co = np.zeros((NBASIS[2], k))
    co[IDX_X2_MINUS_Y2[2], 0] = 1.0
    if k > 1:
        co[:, 1:] = random_coeffs(2, k - 1, data_seed)
    return Workload("c4_2d_p2_jit_%d_k%d" % (m, k), mesh, 2, k, 1e-8, co)


def request_stream(n_requests: int, rate: float, seed: int = 6, max2d: int = 1024,
                   max3d: int = 96, min2d: int = 32, min3d: int = 16, kmax: int = 16):
    """Poisson arrivals of solve requests (mixed serving workload).

    Each request: 2D (p=0.5) with side log-uniform in [min2d, max2d] or 3D with
    side log-uniform in [min3d, max3d]; P1/P2 with p=0.5; structured or jittered
    (0.3h) with p=0.5; k uniform in 1..kmax; random harmonic Dirichlet data.
    Returns a list of dicts with the arrival time and the mesh recipe (meshes
    are built lazily by ``build_request``).
    """
    ua = uniform(seed, STREAM_ARRIVAL, n_requests)
    gaps = -np.log1p(-ua) / rate
    t = np.cumsum(gaps)
    ur = uniform(seed, STREAM_REQUEST, 6 * n_requests).reshape(n_requests, 6)
    reqs = []
    for r in range(n_requests):
        dim = 2 if ur[r, 0] < 0.5 else 3
        lo, hi = (min2d, max2d) if dim == 2 else (min3d, max3d)
        side = int(round(math.exp(math.log(lo) + ur[r, 1] * (math.log(hi) - math.log(lo)))))
        order = 1 if ur[r, 2] < 0.5 else 2
        jit = 0.3 if ur[r, 3] < 0.5 else 0.0
        k = 1 + min(kmax - 1, int(ur[r, 4] * kmax))
        reqs.append(dict(id=r, t_arrival=float(t[r]), dim=dim, m=side, order=order,
                         jitter=jit, k=k, mesh_seed=1000 + r, data_seed=50000 + r))
    return reqs


def build_request(req: dict, tol: float = 1e-8) -> Workload:
    mesh = make_mesh(req["dim"], req["m"], req["jitter"], req["mesh_seed"])
    co = random_coeffs(req["dim"], req["k"], req["data_seed"])
    return Workload("req%d" % req["id"], mesh, req["order"], req["k"], tol, co)
